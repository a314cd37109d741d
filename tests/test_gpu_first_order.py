"""GPU parity of the operator built from first-order perturbative amplitudes
(build_hbar_first_order) with the oracle, and with the general build given the same
amplitudes."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import hbar as ohbar
from oracle import sigma as osig
from oracle import solve as osolve
from paper_1902_06016_amd import gfcc

pytestmark = pytest.mark.gpu


def _first_order_problem(prob):
    """The same problem with T and Lambda replaced by the oracle's first-order amplitudes."""
    t1, t2, l1, l2 = ohbar.first_order_amplitudes(prob.o, prob.v, prob.eps, prob.block("oovv"))
    return t1, t2, l1, l2


@pytest.mark.parametrize("o,v,seed", [(4, 5, 1), (6, 8, 2), (9, 11, 3)])
def test_blocks_sigma_and_solve_match_oracle(gpu_ctx, o, v, seed):
    print(f"[first order o={o} v={v} seed={seed}]", flush=True)
    prob = synth.make_problem(o, v, seed)
    hb = ohbar.build_hbar_first_order(prob)
    gpu_ctx.build_first_order_from_problem(prob)
    for name in ("Foo", "Fov", "Fvv", "Woooo", "Wooov", "Wovvo", "Wovoo"):
        got = gpu_ctx.export(name).cpu().numpy()
        ref = getattr(hb, name)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), name
    diag = gpu_ctx.export("diag").cpu().numpy()
    assert np.abs(diag - osig.diagonal(hb)).max() <= 1e-12 * np.abs(diag).max()
    D = osig.dim(o, v)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((3, D)) + 1j * rng.standard_normal((3, D))
    y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = osig.sigma(hb, x)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    # G and A against dense LU of the first-order operator (c rows with Lambda = T^dagger)
    t1, t2, l1, l2 = _first_order_problem(prob)
    H = osolve.dense_hbar(hb)
    ps = np.arange(o)
    B = np.stack([osig.b_vector(o, v, q) for q in ps], 1)
    C = np.stack([osig.c_vector(o, v, t1, t2, l1, l2, q) for q in ps], 0)
    om = np.linspace(-1.2, -0.3, 7)
    Gd = osolve.green(C, osolve.dense_solve(H, om, B, 0.01))
    res = gpu_ctx.gfcc_solve(om, ps, 0.01, tol=1e-12)
    G = res.G.cpu().numpy()
    assert np.abs(G - Gd).max() <= 1e-10 * np.abs(Gd).max()


def test_same_operator_as_the_general_build(gpu_ctx):
    """The device forms the amplitudes with the oracle's order of operations, so the general
    build fed the oracle's first-order amplitudes gives the same bits."""
    print("[first order vs general build]", flush=True)
    prob = synth.make_problem(7, 9, 5)
    t1, t2, l1, l2 = _first_order_problem(prob)
    D = osig.dim(7, 9)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.standard_normal((5, D)) + 1j * rng.standard_normal((5, D))).cuda()
    gpu_ctx.build_first_order_from_problem(prob)
    y1 = gpu_ctx.sigma_apply(x)
    blocks1 = {n: gpu_ctx.export(n) for n in ("Foo", "Wovvo", "Wovoo", "diag")}
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    gpu_ctx.build_hbar_operands(prob.o, prob.v, dev(prob.eps), dev(t1), dev(t2), dev(l1), dev(l2),
                                *[dev(prob.block(k)) for k in ("oooo", "ooov", "oovv", "ovvo",
                                                              "ovvv")])
    y2 = gpu_ctx.sigma_apply(x)
    assert torch.equal(y1, y2)
    for n, b in blocks1.items():
        assert torch.equal(b, gpu_ctx.export(n)), n


def test_rejects_vanishing_denominators(gpu_ctx):
    print("[first order errors]", flush=True)
    prob = synth.make_problem(4, 5, 1)
    eps = prob.eps.copy()
    eps[3] = eps[4] + 0.1          # highest occupied above the lowest virtual
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    arrs = [dev(eps)] + [dev(prob.block(k)) for k in ("oooo", "ooov", "oovv", "ovvo", "ovvv")]
    st = gfcc.lib.build_hbar_first_order(gpu_ctx.h, 4, 5, *[a.data_ptr() for a in arrs],
                                         gfcc.KEEP_FP64)
    assert st == gfcc.GFCC_EINVAL
    assert b"below every virtual" in gfcc.lib.gfcc_last_error(gpu_ctx.h)
    st = gfcc.lib.build_hbar_first_order(gpu_ctx.h, 4, 5, arrs[0].data_ptr(), None,
                                         *[a.data_ptr() for a in arrs[2:]], gfcc.KEEP_FP64)
    assert st == gfcc.GFCC_EINVAL
