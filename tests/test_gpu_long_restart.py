"""Restart lengths between 33 and 64: every Arnoldi step still runs with delayed
reorthogonalisation, each pass over more than 32 basis vectors split into two sweeps. Checked
against the oracle (dense LU on the small operator; the oracle's sigma for the residual of
returned solutions on a larger one), on both the flow that reads the convergence flags one step
late (small blocks) and the one that finalises each column before the next product (large
blocks), with cycles that go past 32 steps and end early or at the restart length."""
import numpy as np
import pytest

import synth
from oracle import hbar as ohbar
from oracle import sigma as osig
from oracle import solve as osolve
from paper_1902_06016_amd import gfcc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("restart,transpose", [(40, False), (64, False), (48, True), (65, False)])
def test_small_blocks_against_dense_lu(gpu_ctx, restart, transpose):
    """o=10, v=20 next to the 1h poles (about 40 to 60 iterations at tol 1e-12): restart 40 and
    48 stop inside the split range, 64 runs to it, 65 takes the CGS2 path beyond it."""
    print(f"[long restart small restart={restart} T={transpose}]", flush=True)
    o, v, eta = 10, 20, 0.01
    prob = synth.make_problem(o, v, 0)
    hb = ohbar.build_hbar_from_problem(prob)
    dg = osig.diagonal(hb)
    om = np.concatenate([-dg[o - 1] + np.array([-3e-3, 2e-3, 6e-3]),
                         -dg[o - 3] + np.array([-4e-3, 5e-3]), np.linspace(-1.0, -0.3, 7)])
    ps = np.array([o - 4, o - 3, o - 2, o - 1], dtype=np.int32)
    keep = gfcc.KEEP_FP64 | (gfcc.KEEP_TRANSPOSE if transpose else 0)
    gpu_ctx.build_from_problem(prob, keep=keep)
    res = gpu_ctx.gfcc_solve(om, ps, eta, tol=1e-12, restart=restart, maxit=2000,
                             transpose=transpose, want_x=True)
    print(f"  iterations {res.iters.min()}..{res.iters.max()}", flush=True)
    assert res.resid.max() <= 1e-12
    assert res.iters.max() > 33, "the case must reach the split sweeps"
    H = osolve.dense_hbar(hb)
    if transpose:  # (omega - i eta + Hbar_N)^T Y = c_p
        C = np.stack([osig.c_vector(o, v, prob.t1, prob.t2, prob.l1, prob.l2, int(q))
                      for q in ps], 0)
        Xr = np.stack([np.linalg.solve(osolve.shifted(H, w, eta).T, C.T.astype(complex)).T
                       for w in om])
    else:
        B = np.stack([osig.b_vector(o, v, int(p)) for p in ps], 1)
        Xr = osolve.dense_solve(H, om, B, eta)  # [nw][np][D]
    X = res.X.cpu().numpy()
    err = np.abs(X - Xr).max() / np.abs(Xr).max()
    assert err < 1e-9, err
    # the same block with graph capture: eager, captured, replayed steps give the same bits
    try:
        gpu_ctx.graphs(False)
        ref = gpu_ctx.gfcc_solve(om, ps, eta, tol=1e-12, restart=restart, maxit=2000,
                                 transpose=transpose, want_x=True)
        gpu_ctx.graphs(True)
        for rep in range(3):
            r = gpu_ctx.gfcc_solve(om, ps, eta, tol=1e-12, restart=restart, maxit=2000,
                                   transpose=transpose, want_x=True)
            assert np.array_equal(r.X.cpu().numpy(), ref.X.cpu().numpy()), rep
            assert np.array_equal(r.iters, ref.iters), rep
    finally:
        gpu_ctx.graphs(True)


@pytest.mark.parametrize("restart", [48, 36])
def test_large_block_against_oracle_residual(gpu_ctx, restart):
    """o=20, v=50 (D = 9520): 256 right-hand sides in one block take the flow that finalises
    each column before the next product. Frequencies just above the 1h pole of the highest
    occupied orbital take 33 to 39 steps of unrestarted GMRES at tol 1e-10 (the oracle's count):
    at restart 48 every column stops inside the split range and the cycle ends there early; at
    restart 36 the cycle runs to its end (a split final sweep) and the columns left go on after
    the restart. The returned solutions' residuals are formed with the oracle's sigma at the
    hardest columns, and G agrees with the solve at restart 30 (unsplit sweeps) to the
    tolerance."""
    print(f"[long restart large block o20v50 restart={restart}]", flush=True)
    o, v, eta = 20, 50, 0.005
    prob = synth.make_problem(o, v, 7)
    hb = ohbar.build_hbar_from_problem(prob)
    dg = osig.diagonal(hb)
    ps = synth.valence_p(o, 8)
    gpu_ctx.build_from_problem(prob)
    om = np.linspace(-dg[o - 1] - 0.4, -dg[o - 1] + 0.1, 32)
    tol = 1e-10
    res = gpu_ctx.gfcc_solve(om, ps, eta, tol=tol, restart=restart, block=256, maxit=3000,
                             want_x=True)
    print(f"  iterations {res.iters.min()}..{res.iters.max()}", flush=True)
    assert res.resid.max() <= tol
    assert res.iters.max() > 33
    if restart < 40:
        assert res.iters.max() > restart, "the case must restart"
    r30 = gpu_ctx.gfcc_solve(om, ps, eta, tol=tol, restart=30, block=256, maxit=3000)
    G, G30 = res.G.cpu().numpy(), r30.G.cpu().numpy()
    assert np.abs(G - G30).max() <= 1e-8 * np.abs(G30).max()
    X = res.X.cpu().numpy()
    op = osolve.Operator(hb)
    hard = np.unravel_index(np.argsort(res.iters, axis=None)[::-1], res.iters.shape)
    for w, k in [(hard[0][0], hard[1][0]), (hard[0][1], hard[1][1]), (0, 0)]:
        b = osig.b_vector(o, v, int(ps[k]))
        xr = X[w, k]
        z = om[w] - 1j * eta
        hx = op.hbar(xr)
        true = np.linalg.norm(b - (hx + z * xr)) / np.linalg.norm(b)
        # rounding of H x between the two operators' summation orders (see the near-pole test)
        fl = np.finfo(float).eps * (np.linalg.norm(hx) + abs(z) * np.linalg.norm(xr)) \
            / np.linalg.norm(b)
        print(f"  omega={om[w]:.4f} p={ps[k]} its {res.iters[w, k]}: residual "
              f"{res.resid[w, k]:.2e} vs oracle {true:.2e} (rounding scale {fl:.1e})", flush=True)
        assert abs(true - res.resid[w, k]) <= 1e-13 + 16 * fl
        assert true <= tol + 16 * fl


@pytest.mark.parametrize("restart,prec", [(33, gfcc.FP64), (48, gfcc.FP32), (48, gfcc.BF16_PAIRS)])
def test_smallest_split_and_reduced_precision(gpu_ctx, restart, prec):
    """Restart 33: every split has a single earlier basis vector (c = 1). Reduced-precision
    GMRES-IR at restart 48: the inner cycles run the split sweeps on vectors whose sigma comes
    in FP32 (or bf16 pairs), every cycle restarts from the explicit FP64 residual, and the
    scratch vector of the split update sweep is that residual's buffer between restarts. Small
    case next to the 1h poles, against dense LU (tol 1e-10 on the FP64 residual)."""
    print(f"[long restart restart={restart} prec={prec}]", flush=True)
    o, v, eta = 10, 20, 0.01
    prob = synth.make_problem(o, v, 0)
    hb = ohbar.build_hbar_from_problem(prob)
    dg = osig.diagonal(hb)
    om = np.concatenate([-dg[o - 1] + np.array([-3e-3, 2e-3, 6e-3]), np.linspace(-1.0, -0.3, 5)])
    ps = np.array([o - 3, o - 2, o - 1], dtype=np.int32)
    keep = gfcc.KEEP_FP64 | (gfcc.KEEP_FP32 if prec != gfcc.FP64 else 0)
    gpu_ctx.build_from_problem(prob, keep=keep)
    res = gpu_ctx.gfcc_solve(om, ps, eta, tol=1e-10, restart=restart, maxit=3000,
                             precision=prec, want_x=True)
    print(f"  iterations {res.iters.min()}..{res.iters.max()}", flush=True)
    assert res.resid.max() <= 1e-10
    assert res.iters.max() > 33
    H = osolve.dense_hbar(hb)
    B = np.stack([osig.b_vector(o, v, int(p)) for p in ps], 1)
    Xr = osolve.dense_solve(H, om, B, eta)
    err = np.abs(res.X.cpu().numpy() - Xr).max() / np.abs(Xr).max()
    assert err < 1e-7, err
