"""GPU parity: reduced-order model, mixed-precision refinement and the adjoint gradient."""
import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
from oracle import hbar as ohbar
from oracle import mor as omor
from oracle import sigma as osig
from oracle import solve as osolve
from paper_1902_06016_amd import gfcc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model():
    o, v = 6, 10
    p = synth.make_problem(o, v, 31)
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    lam = np.sort(np.linalg.eigvals(H).real)
    ps = np.array([o - 2, o - 1])
    B = np.stack([osig.b_vector(o, v, q) for q in ps], 1)
    C = np.stack([osig.c_vector(o, v, p.t1, p.t2, p.l1, p.l2, q) for q in ps], 0)
    return p, hb, H, lam, ps, B, C


def test_mor_matches_oracle_model(gpu_ctx, model):
    print("[mor_vs_oracle]", flush=True)
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    wk = np.linspace(-lam[0] - 0.3, -lam[0] + 0.3, 3)
    gpu_ctx.build_from_problem(p)
    m = gpu_ctx.mor_build(wk, ps, eta, solve_tol=1e-13, defl_tol=1e-10)
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend(wk, 1e-10)
    order, oks = m.info()
    assert order == rom.m and np.allclose(oks, wk)
    grid = np.linspace(-lam[0] - 0.5, -lam[0] + 0.5, 41)
    Gg, rg = m.eval(grid)
    Go, ro = rom.eval(grid)
    Gg = Gg.cpu().numpy()
    assert np.abs(Gg - Go).max() < 1e-9 * np.abs(Go).max()
    assert np.abs(rg - ro).max() < 1e-7
    # interpolation at the sampled frequencies (Eq. model and the text after it)
    Gk, rk = m.eval(wk)
    Gfull = osolve.green(C, osolve.dense_solve(H, wk, B, eta))
    assert np.abs(Gk.cpu().numpy() - Gfull).max() < 1e-10 * np.abs(Gfull).max()
    assert rk.max() < 1e-9
    m.close()


@pytest.mark.parametrize("nq", [7, 9])
def test_mor_both_reduced_solvers(gpu_ctx, nq):
    """Orders 56 and 72 (o=9, v=16, 4 sampled frequencies): the first fits one wavefront's LDS,
    the second runs on the workgroup-per-frequency solver. Both give the oracle's model,
    residuals and lifted solutions. The frequencies are spread so that every column's
    remainder after orthogonalisation stays above 1.5e-6 of its norm, far from the 1e-10
    deflation threshold (with densely sampled frequencies many remainders fall near the
    threshold and the order then depends on solver rounding: GMRES here, dense LU in the
    oracle)."""
    print(f"[mor_orders nq={nq}]", flush=True)
    o, v, nk = 9, 16, 4
    p = synth.make_problem(o, v, 4)
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    lam0 = np.sort(np.linalg.eigvals(H).real)[0]
    ps = np.arange(o - nq, o)
    B = np.stack([osig.b_vector(o, v, q) for q in ps], 1)
    C = np.stack([osig.c_vector(o, v, p.t1, p.t2, p.l1, p.l2, q) for q in ps], 0)
    eta = 0.01
    wk = np.linspace(-lam0 - 1.2, -lam0 + 1.0, nk)
    gpu_ctx.build_from_problem(p)
    m = gpu_ctx.mor_build(wk, ps, eta, solve_tol=1e-12, defl_tol=1e-10)
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend(wk, 1e-10)
    order, _ = m.info()
    assert order == rom.m == 2 * nq * nk
    grid = np.linspace(-lam0 - 1.4, -lam0 + 1.2, 57)
    Gg, rg = m.eval(grid)
    Go, ro = rom.eval(grid)
    # The basis comes from GMRES solutions at relative residual 1e-12 (dense LU in the
    # oracle). Next to a pole the model's values carry that error amplified by up to
    # ||M|| / eta ~ 1e3, and the residual estimate moves with the basis directions.
    assert np.abs(Gg.cpu().numpy() - Go).max() < 1e-8 * np.abs(Go).max()
    assert np.all(np.abs(rg - ro) <= 1e-5 * ro + 1e-9)
    Xg = m.lift(grid[::7]).cpu().numpy()
    Xo = omor.lift(rom, grid[::7])
    assert np.abs(Xg - Xo).max() < 1e-8 * np.abs(Xo).max()
    m.close()


def test_mor_smallest_models(gpu_ctx, model):
    """One sampled frequency: order 2 (Re and Im of one solution) and 4 (two orbitals), the
    smallest reduced systems the wavefront solver meets, against the oracle's model."""
    print("[mor smallest]", flush=True)
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    gpu_ctx.build_from_problem(p)
    grid = np.linspace(-lam[0] - 0.3, -lam[0] + 0.3, 13)
    for cols in ([1], [0, 1]):
        wk = np.array([-lam[0] + 0.1])
        m = gpu_ctx.mor_build(wk, ps[cols], eta, solve_tol=1e-13)
        rom = omor.ROM(hb, ps[cols], eta, C[cols], omor.dense_solver(H, B[:, cols], eta))
        rom.extend(wk, 1e-10)
        assert m.info()[0] == rom.m == 2 * len(cols)
        Gg, rg = m.eval(grid)
        Go, ro = rom.eval(grid)
        assert np.abs(Gg.cpu().numpy() - Go).max() < 1e-10 * np.abs(Go).max()
        assert np.all(np.abs(rg - ro) <= 1e-8 * ro + 1e-12)
        m.close()


def test_mor_refinement(gpu_ctx, model):
    print("[mor_refine]", flush=True)
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    lo, hi = -lam[0] - 0.4, -lam[0] + 0.2
    gpu_ctx.build_from_problem(p)
    m = gpu_ctx.mor_build(np.linspace(lo, hi, 3), ps, eta, solve_tol=1e-12)
    grid = np.linspace(lo - 0.1, hi + 0.1, 161)
    rounds, rmax = m.refine(grid, lo, hi, per_round=2, resid_tol=1e-6)
    assert rmax <= 1e-6 and rounds >= 1
    win = grid[(grid >= lo) & (grid <= hi)]
    Gh, res = m.eval(win)
    assert res.max() <= 1e-6
    G = osolve.green(C, osolve.dense_solve(H, win, B, eta))
    assert np.abs(Gh.cpu().numpy() - G).max() < 1e-4 * np.abs(G).max()
    m.close()


@pytest.mark.parametrize("prec", [gfcc.FP32, gfcc.FP32_BF16_3BODY, gfcc.BF16_PAIRS])
def test_mixed_precision_solve(gpu_ctx, prec):
    print(f"[mixed prec={prec}]", flush=True)
    cfg = synth.WORKLOADS["o10v20"]
    p = synth.make_problem(cfg["o"], cfg["v"], cfg["seed"])
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    om = synth.omega_grid(cfg["omega"])
    ps = synth.valence_p(cfg["o"], cfg["np"])
    B = np.stack([osig.b_vector(p.o, p.v, q) for q in ps], 1)
    C = np.stack([osig.c_vector(p.o, p.v, p.t1, p.t2, p.l1, p.l2, q) for q in ps], 0)
    Ar = osolve.spectral(osolve.green(C, osolve.dense_solve(H, om, B, cfg["eta"])))
    gpu_ctx.build_from_problem(p, keep=gfcc.KEEP_FP32)
    res = gpu_ctx.gfcc_solve(om, ps, cfg["eta"], tol=1e-8, precision=prec)
    assert res.resid.max() <= 1e-8
    A = gfcc.spectral_function(res.G)
    assert np.abs(A - Ar).max() / np.abs(Ar).max() < 1e-6


def test_bf16_pairs_solve_takes_the_pair_kernel(gpu_ctx):
    """GFCC_BF16_PAIRS at a shape the two-term bf16 ovvo kernel handles (v = 40 >= 32, a block
    of 64 right-hand sides, 128 real columns), next to the lowest pole, against dense LU: the
    kernel's launch count (timer 2) shows that it ran, and A is within 1e-6 of the oracle."""
    print("[pairs on the pair kernel]", flush=True)
    o, v = 10, 40
    p = synth.make_problem(o, v, 7)
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    lam0 = np.sort(np.linalg.eigvals(H).real)[0]
    om = np.linspace(-lam0 - 0.3, -lam0 + 0.3, 32)
    ps = np.array([o - 2, o - 1])
    eta = 0.01
    B = np.stack([osig.b_vector(o, v, q) for q in ps], 1)
    C = np.stack([osig.c_vector(o, v, p.t1, p.t2, p.l1, p.l2, q) for q in ps], 0)
    Gr = osolve.green(C, osolve.dense_solve(H, om, B, eta))
    Ar = osolve.spectral(Gr)
    gpu_ctx.build_from_problem(p, keep=gfcc.KEEP_FP32)
    gpu_ctx.timer(2, enable=True, reset=True)
    # the spectrum is dense next to the lowest poles: restarted inner solves take hundreds of
    # iterations here (the oracle's emulation of the same refinement needs 225 at the window's
    # centre), so the iteration cap is generous
    res = gpu_ctx.gfcc_solve(om, ps, eta, tol=1e-8, restart=30, block=64, maxit=4000,
                             precision=gfcc.BF16_PAIRS)
    _, launches = gpu_ctx.timer(2, enable=False, reset=True)
    assert launches > 0
    assert res.resid.max() <= 1e-8 and res.iters.max() > 10
    A = gfcc.spectral_function(res.G)
    assert np.abs(A - Ar).max() / np.abs(Ar).max() < 1e-6
    # the same solve in FP32 never takes the pair kernel
    gpu_ctx.timer(2, enable=True, reset=True)
    gpu_ctx.gfcc_solve(om[:4], ps, eta, tol=1e-8, restart=30, block=64, maxit=4000,
                       precision=gfcc.FP32)
    assert gpu_ctx.timer(2, enable=False, reset=True)[1] == 0


def test_adjoint_gradient(gpu_ctx, model):
    print("[adjoint]", flush=True)
    p, hb, H, lam, ps, B, C = model
    o, v = p.o, p.v
    eta = 0.02
    om = np.linspace(-lam[0] - 0.2, -lam[0] + 0.2, 9)
    w = oadj.trapezoid_weights(om)
    gref = oadj.gradient_dense(H, om, w, B, C, eta, o, v)
    gpu_ctx.build_from_problem(p)
    fwd = gpu_ctx.gfcc_solve(om, ps, eta, tol=1e-13, want_x=True)
    adj = gpu_ctx.gfcc_solve(om, ps, eta, tol=1e-13, transpose=True, want_x=True)
    g = gpu_ctx.gfcc_grad_eps(w, fwd.X, adj.X)
    assert np.abs(g - gref).max() < 1e-9 * np.abs(gref).max()
    # the same through torch.autograd
    from paper_1902_06016_amd.autograd import SpectralWeight
    dev = gpu_ctx.device
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    inputs = dict(t1=up(p.t1), t2=up(p.t2), l1=up(p.l1), l2=up(p.l2), oooo=up(p.block("oooo")),
                  ooov=up(p.block("ooov")), oovv=up(p.block("oovv")), ovvo=up(p.block("ovvo")),
                  ovvv=up(p.block("ovvv")))
    eps = up(p.eps).requires_grad_(True)
    J = SpectralWeight.apply(eps, gpu_ctx, inputs, om, w, ps, eta, 1e-13)
    J.backward()
    assert abs(J.item() - oadj.objective_dense(H, om, w, B, C, eta)) < 1e-10 * abs(J.item())
    assert np.abs(eps.grad.cpu().numpy() - gref).max() < 1e-9 * np.abs(gref).max()
    # central finite differences through the GPU path
    h = 1e-5
    for r in (o - 1, o + 3):
        Js = []
        for s in (1, -1):
            e2 = p.eps.copy()
            e2[r] += s * h
            Js.append(SpectralWeight.apply(up(e2), gpu_ctx, inputs, om, w, ps, eta, 1e-13).item())
        fd = (Js[0] - Js[1]) / (2 * h)
        # relative to the derivative itself, plus the resolution of J's difference at the solve
        # tolerance (1e-13 |J| / h, about 1e-8 here, 1e-7 of the smaller component)
        noise = 1e-13 * abs(J.item()) / h
        assert abs(fd - gref[r]) < 1e-6 * abs(gref[r]) + 10 * noise, (r, fd, gref[r])
