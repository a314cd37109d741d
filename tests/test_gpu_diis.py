"""GPU parity of the complex DIIS solver (gfcc_solve_diis) with the oracle's DIIS: converged
solutions, every micro-iteration of a fixed-length run, residual histories, the adjoint
systems, initial guesses, padding columns and argument errors."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import diis as odiis
from oracle import hbar as ohbar
from oracle import mor as omor
from oracle import sigma as osig
from oracle import solve as osolve
from paper_1902_06016_amd import gfcc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    o, v = 6, 8
    p = synth.make_problem(o, v, 1)
    hb = ohbar.build_hbar_from_problem(p)
    return p, hb


# Tolerances. The iterates agree to ~1e-12 relative: every step is backward stable (QR on the
# GPU, SVD least squares in the oracle). A relative residual formed from them carries an
# absolute rounding error of order eps * ||M|| ||x|| / ||b||, and the extrapolation passes
# differences of that size on to the next cycle. A NumPy replica of the GPU arithmetic,
# compared with the oracle on 84 systems of this operator, differed by at most 1.6e-11 in
# absolute terms and 7e-6 in relative terms; the bound below leaves a margin of 6 and 14.
HIST_RTOL, HIST_ATOL = 1e-4, 1e-10


def hist_close(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and bool(np.all(np.abs(a - b) <= HIST_RTOL * np.abs(b) + HIST_ATOL))


def iters_close(a, b, ndiis):
    """Where a residual ends within rounding of tol, the two sides may stop a few
    micro-iterations apart; they must stop in the same or the next DIIS cycle."""
    d = np.abs(np.asarray(a, dtype=np.int64) - np.asarray(b, dtype=np.int64))
    return int(d.max()) <= ndiis and int(d.sum()) <= 0.02 * int(np.sum(b)) + ndiis


def hist_prefix_close(hg, ho, ndiis):
    n = min(len(hg), len(ho))
    return abs(len(hg) - len(ho)) <= ndiis and hist_close(hg[:n], ho[:n])


def hist_rows(h):
    """GPU history rows up to the -1 padding."""
    out = []
    for row in h.reshape(-1, h.shape[-1]):
        n = int(np.argmax(row < 0)) if (row < 0).any() else len(row)
        out.append(row[:n])
    return out


@pytest.mark.parametrize("block", [0, 4])
def test_converged_solutions_match_oracle(gpu_ctx, small, block):
    print(f"[diis converged block={block}]", flush=True)
    p, hb = small
    om = np.array([-0.9, -0.5, -0.3])
    ps = np.array([0, 3, 5])
    gpu_ctx.build_from_problem(p)
    res = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-12, maxit=400, ndiis=10, block=block,
                                  want_x=True, want_hist=True)
    Xo, its, reso, hists = odiis.solve_points(hb, om, ps, 0.01, tol=1e-12, maxit=400)
    X = res.X.cpu().numpy()
    assert res.resid.max() <= 1e-12
    assert np.abs(X - Xo).max() <= 1e-9 * np.abs(Xo).max()
    # the same number of micro-iterations and the same convergence profile
    assert iters_close(res.iters, its, 10)
    for hg, ho in zip(hist_rows(res.hist), hists):
        assert hist_prefix_close(hg, ho, 10)
    # G = c^T X
    C = np.stack([osig.c_vector(p.o, p.v, p.t1, p.t2, p.l1, p.l2, int(q)) for q in ps], 0)
    Gd = osolve.green(C, Xo)
    assert np.abs(res.G.cpu().numpy() - Gd).max() <= 1e-9 * np.abs(Gd).max()


def test_wide_and_ragged_blocks(gpu_ctx):
    """72 right-hand sides: two 64-lane groups in one block (block 0 -> 72 columns), and
    blocks of 64 whose last one carries 56 padding columns."""
    print("[diis wide]", flush=True)
    o, v = 8, 8
    p = synth.make_problem(o, v, 7)
    hb = ohbar.build_hbar_from_problem(p)
    om = np.linspace(-0.36, -0.2, 9)
    ps = np.arange(o)
    Xo, its, reso, _ = odiis.solve_points(hb, om, ps, 0.01, tol=1e-11, maxit=300)
    gpu_ctx.build_from_problem(p)
    for block in (0, 64):
        res = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-11, maxit=300, block=block,
                                      want_x=True)
        assert res.resid.max() <= 1e-11
        assert iters_close(res.iters, its, 10)
        assert np.abs(res.X.cpu().numpy() - Xo).max() <= 1e-9 * np.abs(Xo).max()


@pytest.mark.parametrize("ndiis,maxit", [(10, 25), (4, 13), (1, 7)])
def test_every_micro_iteration_matches_oracle(gpu_ctx, small, ndiis, maxit):
    """A run cut at maxit (tol unreachable) stops at the same iterate on both sides:
    extrapolations and plain steps compared element by element."""
    print(f"[diis fixed ndiis={ndiis} maxit={maxit}]", flush=True)
    p, hb = small
    om = np.array([-0.95, -0.45])
    ps = np.arange(p.o)
    gpu_ctx.build_from_problem(p)
    res = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-300, maxit=maxit, ndiis=ndiis,
                                  want_x=True, want_hist=True, allow_noconv=True)
    assert res.status == gfcc.GFCC_ENOCONV
    Xo, its, reso, hists = odiis.solve_points(hb, om, ps, 0.01, tol=1e-300, ndiis=ndiis,
                                              maxit=maxit)
    assert (res.iters == maxit).all() and (its == maxit).all()
    X = res.X.cpu().numpy()
    assert np.abs(X - Xo).max() <= 1e-10 * np.abs(Xo).max()
    assert hist_close(res.resid, reso)
    assert hist_close(res.hist.reshape(-1, maxit + 1), np.asarray(hists))


def test_adjoint_systems_match_oracle(gpu_ctx, small):
    print("[diis transpose]", flush=True)
    p, hb = small
    o, v = p.o, p.v
    om = np.array([-0.6, -0.35])
    ps = np.array([1, 4])
    C = np.stack([osig.c_vector(o, v, p.t1, p.t2, p.l1, p.l2, int(q)) for q in ps], 0)
    gpu_ctx.build_from_problem(p)
    res = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-12, maxit=400, transpose=True,
                                  want_x=True)
    Yo, its, _, _ = odiis.solve_points(hb, om, ps, 0.01, tol=1e-12, maxit=400, transpose=True,
                                       rhs=C)
    assert res.resid.max() <= 1e-12
    assert iters_close(res.iters, its, 10)
    assert np.abs(res.X.cpu().numpy() - Yo).max() <= 1e-9 * np.abs(Yo).max()
    # the adjoint systems give the same G as the forward ones
    fwd = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-12, maxit=400)
    Gf, Gt = fwd.G.cpu().numpy(), res.G.cpu().numpy()
    assert np.abs(Gf - Gt).max() <= 1e-9 * np.abs(Gf).max()


def test_initial_guesses(gpu_ctx, small):
    """An exact guess costs no micro-iteration and comes back unchanged; a guess from the
    oracle's reduced model gives the oracle's iterates and fewer micro-iterations."""
    print("[diis x0]", flush=True)
    p, hb = small
    om = np.linspace(-0.7, -0.4, 7)
    ps = np.array([2, 5])
    gpu_ctx.build_from_problem(p)
    ref = gpu_ctx.gfcc_solve(om, ps, 0.01, tol=1e-13, want_x=True)
    res = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-10, want_x=True, x0=ref.X,
                                  want_hist=True)
    assert res.iters.max() == 0 and torch.equal(res.X, ref.X)
    assert (res.hist[..., 0] <= 1e-10).all() and (res.hist[..., 1:] == -1.0).all()
    # guesses: the oracle's two-frequency reduced model lifted to the full space
    H = osolve.dense_hbar(hb)
    B = np.stack([osig.b_vector(p.o, p.v, int(q)) for q in ps], 1)
    C = np.stack([osig.c_vector(p.o, p.v, p.t1, p.t2, p.l1, p.l2, int(q)) for q in ps], 0)
    rom = omor.ROM(hb, ps, 0.01, C, omor.dense_solver(H, B, 0.01))
    rom.extend(np.array([-0.7, -0.4]), 1e-10)
    x0 = omor.lift(rom, om)
    x0_dev = torch.from_numpy(np.ascontiguousarray(x0)).to(gpu_ctx.device)
    guess = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-11, maxit=400, want_x=True, x0=x0_dev)
    plain = gpu_ctx.gfcc_solve_diis(om, ps, 0.01, tol=1e-11, maxit=400)
    Xo, its, _, _ = odiis.solve_points(hb, om, ps, 0.01, tol=1e-11, maxit=400, x0=x0)
    assert guess.resid.max() <= 1e-11
    assert iters_close(guess.iters, its, 10)
    assert np.abs(guess.X.cpu().numpy() - Xo).max() <= 1e-9 * np.abs(Xo).max()
    assert guess.iters.sum() < plain.iters.sum()


def test_diagonal_operator_and_errors(gpu_ctx):
    print("[diis diagonal + errors]", flush=True)
    o, v = 4, 5
    p = synth.make_problem(o, v, 2)
    # T = 0 and V = 0: H-bar_N is diagonal and one Jacobi step solves exactly
    p0 = synth.Problem(o=o, v=v, seed=2, eps=p.eps, t1=np.zeros_like(p.t1),
                       blocks={k: np.zeros_like(p.block(k))
                               for k in ("oooo", "ooov", "oovv", "ovvo", "ovvv")},
                       _t2=np.zeros_like(p.t2))
    gpu_ctx.build_from_problem(p0)
    om = np.array([-0.7, -0.25])
    res = gpu_ctx.gfcc_solve_diis(om, np.arange(o), 0.01, tol=1e-14, want_x=True, want_hist=True)
    assert (res.iters == 1).all() and res.resid.max() <= 1e-15
    X = res.X.cpu().numpy()
    for w in range(2):
        for q in range(o):
            assert X[w, q, q] == pytest.approx(1.0 / (om[w] - p.eps[q] - 0.01j), rel=1e-15)
    assert (res.hist[..., 0] == 1.0).all()
    # argument errors
    G = torch.empty((1, 1, 1), dtype=torch.complex128, device=gpu_ctx.device)
    omc = (ctypes.c_double * 1)(-0.5)
    pc = (ctypes.c_int * 1)(0)
    for nd in (0, 17):
        st = gfcc.lib.gfcc_solve_diis(gpu_ctx.h, 1, omc, 1, pc, 0.01, 1e-10, 50, nd, 0, 0, None,
                                      None, G.data_ptr(), None, None, None)
        assert st == gfcc.GFCC_EINVAL
    X = torch.zeros((1, 1, gpu_ctx.D), dtype=torch.complex128, device=gpu_ctx.device)
    st = gfcc.lib.gfcc_solve_diis(gpu_ctx.h, 1, omc, 1, pc, 0.01, 1e-10, 50, 10, 0, 0,
                                  X.data_ptr(), X.data_ptr(), G.data_ptr(), None, None, None)
    assert st == gfcc.GFCC_EINVAL
    assert b"overlap" in gfcc.lib.gfcc_last_error(gpu_ctx.h)
