"""HIP graph capture of the Arnoldi steps of small blocks: with capture on, a step shape runs
eagerly the first time, is captured the second time and replayed afterwards. Every solve, with
eager work and synchronisations between the replays, gives the bits of the same solve launched
kernel by kernel (same kernels, same arguments, same order); so does the oracle check."""
import numpy as np
import pytest
import torch

import synth
from oracle import hbar as ohbar
from oracle import sigma as osig
from oracle import solve as osolve
from paper_1902_06016_amd import gfcc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("transpose", [False, True])
def test_replayed_steps_match_eager_steps(gpu_ctx, transpose):
    print(f"[graphs transpose={transpose}]", flush=True)
    o, v = 10, 20   # the small case's operator and window: about 27 iterations at restart 30
    prob = synth.make_problem(o, v, 0)
    keep = gfcc.KEEP_FP64 | (gfcc.KEEP_TRANSPOSE if transpose else 0)
    gpu_ctx.build_from_problem(prob, keep=keep)
    om = np.linspace(-1.0, -0.3, 12)
    ps = np.array([o - 3, o - 2, o - 1], dtype=np.int32)
    kw = dict(tol=1e-10, restart=16, block=36, transpose=transpose, want_x=True)
    try:
        gpu_ctx.graphs(False)
        ref = gpu_ctx.gfcc_solve(om, ps, 0.01, **kw)
        G0, X0 = ref.G.cpu().numpy(), ref.X.cpu().numpy()
        assert ref.iters.max() > 16, "the test needs more than one restart cycle"
        gpu_ctx.graphs(True)
        g = torch.Generator(device="cuda").manual_seed(5)
        x = torch.randn((6, gfcc.dim(o, v)), dtype=torch.complex128, device="cuda", generator=g)
        y0 = gpu_ctx.sigma_apply(x).cpu().numpy()
        for rep in range(4):  # eager, capture, replay, replay
            r = gpu_ctx.gfcc_solve(om, ps, 0.01, **kw)
            assert np.array_equal(r.G.cpu().numpy(), G0), rep
            assert np.array_equal(r.X.cpu().numpy(), X0), rep
            assert np.array_equal(r.iters, ref.iters) and np.array_equal(r.resid, ref.resid)
            # eager work on the same stream between the replays
            assert np.array_equal(gpu_ctx.sigma_apply(x).cpu().numpy(), y0)
            torch.cuda.synchronize()
        # another maxit is another step shape (its stopping test differs)
        r = gpu_ctx.gfcc_solve(om, ps, 0.01, maxit=400, **kw)
        assert np.array_equal(r.G.cpu().numpy(), G0)
        # a rebuild of the same shape from other inputs keeps the operator's addresses, so the
        # captured steps stay in use; they must read the new operator
        prob2 = synth.make_problem(o, v, 3)
        gpu_ctx.build_from_problem(prob2, keep=keep)
        r2 = [gpu_ctx.gfcc_solve(om, ps, 0.01, **kw).G.cpu().numpy() for _ in range(2)]
        gpu_ctx.graphs(False)
        e2 = gpu_ctx.gfcc_solve(om, ps, 0.01, **kw).G.cpu().numpy()
        assert not np.array_equal(e2, G0)
        assert np.array_equal(r2[0], e2) and np.array_equal(r2[1], e2)
        gpu_ctx.build_from_problem(prob, keep=keep)
    finally:
        gpu_ctx.graphs(True)
    if transpose:
        return
    # and the oracle: dense LU of the same systems
    hb = ohbar.build_hbar_from_problem(prob)
    H = osolve.dense_hbar(hb)
    B = np.stack([osig.b_vector(o, v, p) for p in ps], 1)
    Xd = osolve.dense_solve(H, om, B, 0.01)  # [nw][np][D]
    err = np.abs(X0 - Xd).max() / np.abs(Xd).max()
    assert err < 1e-8, err


def test_graph_switch_errors(gpu_ctx):
    with pytest.raises(gfcc.GfccError):
        gpu_ctx.graphs(2)
    gpu_ctx.graphs(True)
