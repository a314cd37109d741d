"""Restart compaction of GMRES blocks (gfcc_compact): right-hand sides that a restart leaves
active go on in a block of only their columns. Solutions, G and residuals match the dense
oracle and the uncompacted solve, forward and transposed, with a start iterate, and when a
compacted block compacts again."""
import numpy as np
import pytest
import torch

import synth
from oracle import hbar as ohbar
from oracle import sigma as osig
from oracle import solve as osolve

pytestmark = pytest.mark.gpu


def _dense(prob, om, ps, eta, transpose=False):
    hb = ohbar.build_hbar_from_problem(prob)
    H = osolve.dense_hbar(hb)
    o, v = prob.o, prob.v
    if transpose:
        C = np.stack([osig.c_vector(o, v, prob.t1, prob.t2, prob.l1, prob.l2, q) for q in ps], 1)
        return osolve.dense_solve(H.T, om, C, eta)
    B = np.stack([osig.b_vector(o, v, p) for p in ps], 1)
    return osolve.dense_solve(H, om, B, eta)


def _both(ctx, *args, **kw):
    out = []
    for on in (False, True):
        ctx.compact(on)
        out.append(ctx.gfcc_solve(*args, **kw))
    ctx.compact(True)
    return out


@pytest.mark.parametrize("restart,transpose", [(30, False), (8, False), (12, True)])
def test_compacted_restarts_match_oracle(gpu_ctx, restart, transpose):
    """o=10, v=20, 64 omega x 10 p in one block of 640: at restart 30 about a tenth of the
    systems need a second cycle (one compaction to 128 columns); at restart 8 compaction comes
    after several cycles and the compacted block compacts again."""
    print(f"[compact restart={restart} T={transpose}]", flush=True)
    cfg = synth.WORKLOADS["o10v20"]
    prob = synth.make_problem(cfg["o"], cfg["v"], cfg["seed"])
    om = synth.omega_grid(cfg["omega"])
    ps = synth.valence_p(cfg["o"], cfg["np"])
    Xr = _dense(prob, om, ps, cfg["eta"], transpose)
    gpu_ctx.build_from_problem(prob)
    tol = 1e-10
    off, on = _both(gpu_ctx, om, ps, cfg["eta"], tol=tol, restart=restart, block=640,
                    maxit=400, want_x=True, transpose=transpose)
    assert on.iters.max() > restart, "no restart happened"
    scale = np.abs(Xr).max()
    for r in (off, on):
        assert r.resid.max() <= tol
        assert np.abs(r.X.cpu().numpy() - Xr).max() / scale < 1e-8
    # the same iterates up to rounding: counts agree but where a residual sits at the tolerance
    diff = np.abs(on.iters.astype(int) - off.iters.astype(int))
    assert diff.max() <= 2 and (diff > 0).sum() <= 32
    G0, G1 = off.G.cpu().numpy(), on.G.cpu().numpy()
    assert np.abs(G1 - G0).max() / np.abs(G0).max() < 1e-9


def test_compacted_restart_from_a_start_iterate(gpu_ctx):
    """gfcc_solve_x0 from a perturbed dense solution: the first cycle starts from the explicit
    residual, later restarts compact."""
    print("[compact x0]", flush=True)
    cfg = synth.WORKLOADS["o10v20"]
    prob = synth.make_problem(cfg["o"], cfg["v"], cfg["seed"])
    om = synth.omega_grid(cfg["omega"])
    ps = synth.valence_p(cfg["o"], cfg["np"])
    Xr = _dense(prob, om, ps, cfg["eta"])
    gpu_ctx.build_from_problem(prob)
    rng = np.random.default_rng(3)
    x0 = Xr * (1.0 + 1e-3 * rng.standard_normal(Xr.shape))
    # [nw][np][D] as the binding takes it
    x0 = np.ascontiguousarray(x0.reshape(len(om), len(ps), -1))
    x0t = torch.from_numpy(x0).cuda()
    res = []
    for on in (False, True):
        gpu_ctx.compact(on)
        res.append(gpu_ctx.gfcc_solve(om, ps, cfg["eta"], tol=1e-12, restart=6, block=640,
                                      maxit=400, want_x=True, x0=x0t))
    gpu_ctx.compact(True)
    for r in res:
        assert r.resid.max() <= 1e-12
        assert np.abs(r.X.cpu().numpy().reshape(Xr.shape) - Xr).max() / np.abs(Xr).max() < 1e-10
    assert res[1].iters.max() > 6


def test_compacted_blocks_share_captured_steps(gpu_ctx):
    """A compacted block of 128 columns is laid out as a first-level block of 128 columns, so
    the two share captured steps (same step shapes past step 0). Interleaving both kinds of
    solve with graph capture on (eager, capture, replay) gives the bits of the same solves run
    kernel by kernel."""
    print("[compact graphs]", flush=True)
    cfg = synth.WORKLOADS["o10v20"]
    prob = synth.make_problem(cfg["o"], cfg["v"], cfg["seed"])
    om = synth.omega_grid(cfg["omega"])
    ps = synth.valence_p(cfg["o"], cfg["np"])
    gpu_ctx.build_from_problem(prob)
    kw = dict(tol=1e-10, restart=30, maxit=400)

    def pair():
        a = gpu_ctx.gfcc_solve(om, ps[:2], cfg["eta"], block=128, **kw)   # 128 columns
        b = gpu_ctx.gfcc_solve(om, ps, cfg["eta"], block=640, **kw)       # compacts to 128
        return a, b

    try:
        gpu_ctx.graphs(False)
        ra, rb = pair()
        assert rb.iters.max() > 30
        gpu_ctx.graphs(True)
        for rep in range(3):
            a, b = pair()
            for x, y in ((a, ra), (b, rb)):
                assert np.array_equal(x.G.cpu().numpy(), y.G.cpu().numpy()), rep
                assert np.array_equal(x.iters, y.iters) and np.array_equal(x.resid, y.resid)
    finally:
        gpu_ctx.graphs(True)
