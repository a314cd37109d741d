"""GPU tests of the solver's failure paths that the host can force (an exactly singular shifted
operator), of the undamped limit eta = 0, of the windowed spectral weight, and of the
independence of the (omega, p) systems: a system's result does not depend on which other
systems share its block."""
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


def _up(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _build(ctx, o, v, eps, t1=None, t2=None, oooo=None, ooov=None, oovv=None, ovvo=None,
           ovvv=None):
    z = lambda *s: np.zeros(s)  # noqa: E731
    t1 = z(o, v) if t1 is None else t1
    t2 = z(o, o, v, v) if t2 is None else t2
    arrs = [eps, t1, t2, t1, t2,
            z(o, o, o, o) if oooo is None else oooo, z(o, o, o, v) if ooov is None else ooov,
            z(o, o, v, v) if oovv is None else oovv, z(o, v, v, o) if ovvo is None else ovvo,
            z(o, v, v, v) if ovvv is None else ovvv]
    ctx.build_hbar_operands(o, v, *[_up(a) for a in arrs])
    torch.cuda.synchronize()


def _solve_raw(ctx, omega, ps, eta, tol=1e-12, maxit=50, restart=30):
    """gfcc_solve through the C ABI, returning the status instead of raising."""
    om = np.ascontiguousarray(omega, dtype=np.float64)
    pp = np.ascontiguousarray(ps, dtype=np.int32)
    nw, np_ = len(om), len(pp)
    G = torch.full((nw, np_, np_), np.nan, dtype=torch.complex128, device="cuda")
    its = np.full(nw * np_, -7, dtype=np.int32)
    res = np.full(nw * np_, -7.0)
    st = gfcc.lib.gfcc_solve(ctx.h, nw, om.ctypes.data_as(ctypes.c_void_p), np_,
                             pp.ctypes.data_as(ctypes.c_void_p), eta, tol, maxit, restart, 0,
                             gfcc.FP64, 0, None, ctypes.c_void_p(G.data_ptr()),
                             its.ctypes.data_as(ctypes.c_void_p),
                             res.ctypes.data_as(ctypes.c_void_p))
    return st, G.cpu().numpy(), its.reshape(nw, np_), res.reshape(nw, np_)


def test_zero_diagonal_without_broadening(gpu_ctx):
    """T = V = 0 and eta = 0: the shifted operator is diagonal, and exactly singular at
    omega = eps_i (a pole). The solve reports EBREAKDOWN before any iteration and leaves the
    outputs alone; off the poles it returns the closed form G_ii = 1/(omega - eps_i)."""
    print("[eta=0 diagonal]", flush=True)
    o, v = 3, 2
    eps = np.array([-1.25, -0.75, -0.5, 0.5, 1.5])
    _build(gpu_ctx, o, v, eps)
    ps = np.arange(o)
    st, G, its, res = _solve_raw(gpu_ctx, [-0.3, -0.75], ps, 0.0)
    assert st == gfcc.GFCC_EBREAKDOWN
    assert np.isnan(G).all() and (its == -7).all()
    assert "omega" in gfcc.lib.gfcc_last_error(gpu_ctx.h).decode()
    om = np.array([-0.3, -1.0, 0.25])
    st, G, its, res = _solve_raw(gpu_ctx, om, ps, 0.0)
    assert st == gfcc.GFCC_OK and res.max() <= 1e-12
    for w in range(len(om)):
        assert np.abs(np.diag(G[w]) - 1.0 / (om[w] - eps[:o])).max() <= 1e-14 * np.abs(
            1.0 / (om[w] - eps[:o])).max()
    # negative broadening is still an argument error
    with pytest.raises(gfcc.GfccError) as e:
        gpu_ctx.gfcc_solve([-0.3], [0], -1e-3)
    assert e.value.status == gfcc.GFCC_EINVAL


def test_singular_on_a_krylov_space(gpu_ctx):
    """o = 2, v = 1 (D = 3) with T = 0, eps = -1 and <01||0a> = -1: Hbar_N (checked against the
    oracle) is [[1,0,1],[0,1,0],[1,0,1]], so at omega = 0, eta = 0 the shifted operator is
    singular with a unit diagonal. GMRES from b = e_0 meets a zero pivot in its second step
    (the Krylov space {e_0, e_2} is invariant and M restricted to it is singular): EBREAKDOWN,
    with the other orbital's system (b = e_1, an eigenvector) solved in one step."""
    print("[krylov breakdown]", flush=True)
    o, v = 2, 1
    eps = np.array([-1.0, -1.0, -1.0])
    ooov = np.zeros((o, o, o, v))
    ooov[0, 1, 0, 0], ooov[1, 0, 0, 0] = -1.0, 1.0
    z = lambda *s: np.zeros(s)  # noqa: E731
    hb = ohbar.build_hbar(o, v, eps, z(o, v), z(o, o, v, v), z(o, o, o, o), ooov,
                          z(o, o, v, v), z(o, v, v, o), z(o, v, v, v))
    H = osolve.dense_hbar(hb)
    assert np.array_equal(H, np.array([[1.0, 0, 1], [0, 1, 0], [1, 0, 1]]))
    _build(gpu_ctx, o, v, eps, ooov=ooov)
    st, G, its, res = _solve_raw(gpu_ctx, [0.0], [0, 1], 0.0)
    assert st == gfcc.GFCC_EBREAKDOWN, gfcc.lib.gfcc_last_error(gpu_ctx.h)
    assert its[0, 0] == 2 and np.isfinite(res[0, 0]) and res[0, 0] > 0.1
    assert its[0, 1] == 1 and res[0, 1] <= 1e-15
    assert G[0, 1, 1] == 1.0 and np.isfinite(G).all()
    # with broadening the same operator is regular and the solve matches the dense one
    st, G, its, res = _solve_raw(gpu_ctx, [0.0], [0, 1], 0.25)
    assert st == gfcc.GFCC_OK
    X = np.linalg.solve(H + (0.0 - 0.25j) * np.eye(3), np.eye(3)[:, :2].astype(complex))
    assert np.abs(np.diag(G[0]) - np.diag(X[:2, :2])).max() < 1e-14


def test_undamped_solve_matches_dense(gpu_ctx):
    """eta = 0 off the poles: real shifted systems, against dense LU."""
    print("[eta=0 dense]", flush=True)
    prob = synth.make_problem(6, 10, 2)
    hb = ohbar.build_hbar_from_problem(prob)
    H = osolve.dense_hbar(hb)
    lam = np.sort(np.linalg.eigvals(H).real)
    om = np.array([-lam[0] + 0.4, -lam[0] + 0.9])
    ps = np.array([4, 5])
    B = np.stack([osig.b_vector(6, 10, q) for q in ps], 1)
    C = np.stack([osig.c_vector(6, 10, prob.t1, prob.t2, prob.l1, prob.l2, q) for q in ps], 0)
    Gr = osolve.green(C, osolve.dense_solve(H, om, B, 0.0))
    gpu_ctx.build_from_problem(prob)
    res = gpu_ctx.gfcc_solve(om, ps, 0.0, tol=1e-12, maxit=400)
    assert np.abs(res.G.cpu().numpy() - Gr).max() < 1e-10 * np.abs(Gr).max()


def test_spectral_weight(gpu_ctx):
    rng = np.random.default_rng(2)
    G = rng.standard_normal((7, 3, 3)) + 1j * rng.standard_normal((7, 3, 3))
    w = rng.standard_normal(7)
    ref = float(np.dot(w, np.einsum("wpp->w", G.imag))) / np.pi
    assert abs(gfcc.spectral_weight(G, w) - ref) < 1e-14 * np.abs(G).sum()
    assert abs(gfcc.spectral_weight(torch.from_numpy(G).cuda(), w) - ref) < 1e-14 * np.abs(G).sum()
    assert gfcc.spectral_weight(np.zeros((0, 2, 2), dtype=complex), np.zeros(0)) == 0.0
    J = ctypes.c_double()
    assert gfcc.lib.spectral_weight(-1, 1, None, 0, None, ctypes.byref(J)) == gfcc.GFCC_EINVAL
    assert gfcc.lib.spectral_weight(2, 1, None, 0, None, ctypes.byref(J)) == gfcc.GFCC_EINVAL


@pytest.mark.parametrize("transpose", [False, True])
def test_block_layout_independence(gpu_ctx, transpose):
    """The (omega, p) systems are independent: in blocks of one width, a system gets the same
    bits whichever systems share its block and wherever it sits in it (16 frequencies x 8
    orbitals in blocks of 64, against the frequencies interleaved and reversed). Blocks of
    another width change the product shapes and with them the summation order inside the
    library's matrix products, so there the results agree to rounding."""
    print(f"[layout T={transpose}]", flush=True)
    cfg = synth.WORKLOADS["o10v20"]
    prob = synth.make_problem(cfg["o"], cfg["v"], cfg["seed"])
    gpu_ctx.build_from_problem(prob)
    om = synth.omega_grid(cfg["omega"])[::4][:16]
    ps = synth.valence_p(cfg["o"], 8)
    kw = dict(tol=1e-11, restart=20, transpose=transpose, want_x=True)
    a = gpu_ctx.gfcc_solve(om, ps, cfg["eta"], block=64, **kw)
    perm = np.concatenate([np.arange(16)[::2], np.arange(16)[1::2]])[::-1]
    b = gpu_ctx.gfcc_solve(om[perm], ps, cfg["eta"], block=64, **kw)
    inv = np.argsort(perm)
    Ga, Gb = a.G.cpu().numpy(), b.G.cpu().numpy()[inv]
    Xa, Xb = a.X.cpu().numpy(), b.X.cpu().numpy()[inv]
    assert np.array_equal(Ga, Gb) and np.array_equal(Xa, Xb)
    assert np.array_equal(a.iters, b.iters[inv]) and np.array_equal(a.resid, b.resid[inv])
    # the second half alone (one block of 64) against its place in the first call
    c = gpu_ctx.gfcc_solve(om[8:], ps, cfg["eta"], block=64, **kw)
    assert np.array_equal(c.G.cpu().numpy(), Ga[8:]) and np.array_equal(c.X.cpu().numpy(), Xa[8:])
    # one block of 128: other product shapes, the same solutions to the tolerance
    d = gpu_ctx.gfcc_solve(om, ps, cfg["eta"], block=128, **kw)
    assert np.abs(d.G.cpu().numpy() - Ga).max() <= 1e-9 * np.abs(Ga).max()
