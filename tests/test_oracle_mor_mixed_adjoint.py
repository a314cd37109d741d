"""Pins of the oracle's reduced-order model, mixed-precision refinement and adjoint gradient."""
import numpy as np
import pytest

import synth
from oracle import adjoint as oadj
from oracle import hbar as ohbar
from oracle import mixed as omix
from oracle import mor as omor
from oracle import sigma as osig
from oracle import solve as osolve


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


def test_rom_interpolates_at_sampled_frequencies(model):
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    wk = np.linspace(-lam[0] - 0.3, -lam[0] + 0.3, 3)
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend(wk, 1e-12)
    Gh, res = rom.eval(wk)
    G = osolve.green(C, osolve.dense_solve(H, wk, B, eta))
    assert np.abs(Gh - G).max() < 1e-10 * np.abs(G).max()
    assert res.max() < 1e-10
    # between samples the model is an approximation: non-zero residual
    _, res_mid = rom.eval(0.5 * (wk[:-1] + wk[1:]))
    assert res_mid.max() > 1e-8


def test_rom_full_order_is_exact(model):
    p, hb, H, lam, ps, B, C = model
    eta = 0.02
    D = H.shape[0]
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    # any orthonormal basis of the whole space: the reduced model is the full model
    rom.extend([-1.0], 1e-12)
    Q, _ = np.linalg.qr(np.concatenate([rom.S, np.random.default_rng(5).standard_normal((D, D))], 1))
    rom.S = Q[:, :D]
    rom.HS = osig.sigma(hb, rom.S.T).T
    assert rom.m == D
    om = np.linspace(-4, 0, 9)
    Gh, res = rom.eval(om)
    G = osolve.green(C, osolve.dense_solve(H, om, B, eta))
    assert np.abs(Gh - G).max() < 1e-9 * np.abs(G).max()


def test_rom_basis_rotation_invariance(model):
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend(np.linspace(-2.0, -1.0, 3), 1e-12)
    om = np.linspace(-2.2, -0.8, 7)
    G1, r1 = rom.eval(om)
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((rom.m, rom.m)))
    rom.S = rom.S @ Q
    rom.HS = rom.HS @ Q
    G2, r2 = rom.eval(om)
    assert np.abs(G1 - G2).max() < 1e-10 * np.abs(G1).max()
    assert np.abs(r1 - r2).max() < 1e-8


def test_refinement_reaches_threshold(model):
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    lo, hi = -lam[0] - 0.4, -lam[0] + 0.2
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend(np.linspace(lo, hi, 3), 1e-10)
    grid = np.linspace(lo, hi, 121)
    rounds, rmax = omor.refine(rom, grid, lo, hi, 2, 1e-6, 10_000, 50, 1e-10)
    assert rmax <= 1e-6 and rounds >= 1
    G = osolve.green(C, osolve.dense_solve(H, grid, B, eta))
    Gh, _ = rom.eval(grid)
    assert np.abs(Gh - G).max() < 1e-4 * np.abs(G).max()


def test_lift_interpolates_and_carries_the_model_residual(model):
    """S xhat(omega) equals the full solution at sampled frequencies; between them its true
    residual (formed with the dense H-bar) equals the model's residual estimate, and c^T of it
    is the model's Green's function."""
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    wk = np.linspace(-lam[0] - 0.3, -lam[0] + 0.3, 3)
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend(wk, 1e-12)
    Xk = omor.lift(rom, wk)
    Xd = osolve.dense_solve(H, wk, B, eta)
    assert np.abs(Xk - Xd).max() < 1e-10 * np.abs(Xd).max()
    mid = 0.5 * (wk[:-1] + wk[1:])
    Xm = omor.lift(rom, mid)
    Gh, res = rom.eval(mid)
    for w, om in enumerate(mid):
        R = B - osolve.shifted(H, om, eta) @ Xm[w].T
        true = np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0))
        assert abs(true - res[w]) <= 1e-6 * res[w] + 1e-14
        assert np.abs(C @ Xm[w].T - Gh[w]).max() < 1e-10 * np.abs(Gh[w]).max()
    assert res.max() > 1e-8          # a real approximation between samples


def test_per_diagonal_models_sum_to_the_spectral_function(model):
    """One model per diagonal curve G_pp (basis from X_p alone): at the sampled frequencies
    every curve, and so their sum A, is the full one; between them the sum approximates A."""
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    wk = np.linspace(-lam[0] - 0.3, -lam[0] + 0.3, 4)
    grid = np.linspace(wk[0], wk[-1], 25)
    Afull = osolve.spectral(osolve.green(C, osolve.dense_solve(H, grid, B, eta)))
    Ak = osolve.spectral(osolve.green(C, osolve.dense_solve(H, wk, B, eta)))
    curves_k, curves = [], []
    for k, q in enumerate(ps):
        rom = omor.ROM(hb, [q], eta, C[k:k + 1], omor.dense_solver(H, B[:, k:k + 1], eta))
        rom.extend(wk, 1e-12)
        assert rom.m <= 2 * len(wk)
        curves_k.append(rom.eval(wk)[0][:, 0, 0])
        curves.append(rom.eval(grid)[0][:, 0, 0])
    A_k = np.sum(np.imag(curves_k), 0) / np.pi
    A = np.sum(np.imag(curves), 0) / np.pi
    assert np.abs(A_k - Ak).max() < 1e-10 * np.abs(Ak).max()
    err = np.abs(A - Afull).max() / np.abs(Afull).max()
    assert 0 < err < 1e-1


def test_gmres_initial_guess(model):
    """An exact x0 needs no iteration; a reduced-model x0 converges to the same solution in no
    more iterations than x0 = 0."""
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    op = osolve.Operator(hb)
    om = -lam[0] + 0.05
    xd = osolve.dense_solve(H, [om], B, eta)[0, 0]
    x, it, rel = osolve.gmres(op, B[:, 0], om, eta, tol=1e-10, x0=xd)
    assert it == 0 and np.abs(x - xd).max() == 0.0
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend([om - 0.2, om + 0.2], 1e-12)
    x0 = omor.lift(rom, [om])[0, 0]
    x1, it1, rel1 = osolve.gmres(op, B[:, 0], om, eta, tol=1e-10, x0=x0)
    x2, it2, rel2 = osolve.gmres(op, B[:, 0], om, eta, tol=1e-10)
    assert rel1 <= 1e-10 and rel2 <= 1e-10
    assert it1 < it2
    assert np.abs(x1 - xd).max() < 1e-8 * np.abs(xd).max()


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.0e-8, 65504.0], dtype=np.float32)
    r = omix.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0078125)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_bf16_split():
    """Two-term bf16 values: hi is the bf16 rounding, hi + lo recovers x to about 2^-16
    relative, and values that fit two bf16 halves are exact."""
    x = np.array([1.0 + 2.0 ** -10, np.pi, -0.05, 3.0e-7], dtype=np.float64)
    hi, lo = omix.bf16_split(x)
    assert np.array_equal(hi, omix.bf16_round(x.astype(np.float32)))
    assert hi[0] == 1.0 and lo[0] == 2.0 ** -10          # 1 + 2^-10: exact in two halves
    assert hi[1] == np.float32(3.140625)                  # pi: 8 significant bits, then the rest
    err = np.abs(hi.astype(np.float64) + lo - x)
    assert np.all(err <= np.abs(x) * 2.0 ** -16)
    assert np.all(np.abs(lo) <= np.abs(x) * 2.0 ** -8)


def test_bf16_three_body_term_keeps_16_bits(model):
    """The emulated bf16 three-body term (hi.hi + hi.lo + lo.hi in float32) differs from the
    float32 term by about 2^-17 of its size here (bound 2^-14); plain bf16 operands are off by
    about 2^-8.4 and fail the bound."""
    p, hb, H, lam, ps, B, C = model
    rng = np.random.default_rng(3)
    D = osig.dim(p.o, p.v)
    x = rng.standard_normal((4, D)) + 1j * rng.standard_normal((4, D))
    t9 = osig.sigma_parts(hb, x.real)["T9"] + 1j * osig.sigma_parts(hb, x.imag)["T9"]
    h32 = omix.f32_hbar(hb)
    full = omix.sigma_reduced(h32, x, bf16_3body=True)
    plain = omix.sigma_reduced(h32, x, bf16_3body=False)   # float32 throughout
    # the difference between the two reduced forms is the three-body term's bf16 error
    assert np.abs(full - plain).max() <= 2.0 ** -14 * np.abs(t9).max()
    assert np.abs(full - osig.sigma(hb, x)).max() <= 1e-6 * np.abs(osig.sigma(hb, x)).max()


def test_bf16_pair_products_within_their_bound(model):
    """The two-term bf16 forms of the T5, T6 and T8 contractions differ from the FP64 ones by
    at most 2^-14 of sum |a||b| over the contracted index (operand pairs carry 16 bits:
    |lo| <= 2^-8 |x| after round-to-nearest to bf16, so the dropped lo.lo term is at most
    about 2^-16 of a product; float32 accumulation adds K 2^-24 at most);
    plain bf16 operands miss this bound."""
    p, hb, H, lam, ps, B, C = model
    o, v = p.o, p.v
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, osig.dim(o, v)))
    _, r2 = osig.unpack(x, o, v)
    for spec, blk in (("ae,...ije->...ija", hb.Fvv), ("ki,...kja->...ija", hb.Foo),
                      ("maei,...mje->...ija", hb.Wovvo)):
        exact = np.einsum(spec, blk, r2)
        bound = 2.0 ** -14 * np.einsum(spec, np.abs(blk), np.abs(r2))
        got = omix._pair_product(spec, blk.astype(np.float32), r2.astype(np.float32))
        assert np.all(np.abs(got - exact) <= bound), spec
        single = np.einsum(spec, omix.bf16_round(blk), omix.bf16_round(r2))
        assert np.any(np.abs(single - exact) > bound), spec


def test_bf16_pairs_sigma_close_to_fp64(model):
    p, hb, H, lam, ps, B, C = model
    rng = np.random.default_rng(6)
    D = osig.dim(p.o, p.v)
    x = rng.standard_normal((2, D)) + 1j * rng.standard_normal((2, D))
    y = osig.sigma(hb, x)
    got = omix.sigma_reduced(omix.f32_hbar(hb), x, bf16_3body=False, pairs=True)
    assert np.abs(got - y).max() <= 1e-4 * np.abs(y).max()


def test_gmres_ir_reaches_fp64_tolerance(model):
    p, hb, H, lam, ps, B, C = model
    om, eta = -lam[0] + 0.05, 0.005
    xd = np.linalg.solve(osolve.shifted(H, om, eta), B[:, 1].astype(complex))
    for pairs in (False, True):
        x, outer, inner, rel = omix.gmres_ir(hb, B[:, 1].astype(complex), om, eta, tol=1e-10,
                                             bf16_3body=not pairs, pairs=pairs)
        assert rel <= 1e-10 and outer >= 2
        assert np.abs(x - xd).max() < 1e-8 * np.abs(xd).max()


def test_adjoint_gradient_matches_finite_differences(model):
    p, hb, H, lam, ps, B, C = model
    o, v = p.o, p.v
    eta = 0.02
    om = np.linspace(-lam[0] - 0.2, -lam[0] + 0.2, 9)
    w = oadj.trapezoid_weights(om)
    g = oadj.gradient_dense(H, om, w, B, C, eta, o, v)
    h = 1e-5
    for r in (0, o - 1, o + 2):
        ep, em = p.eps.copy(), p.eps.copy()
        ep[r] += h
        em[r] -= h
        Jp = oadj.objective_dense(osolve.dense_hbar(oadj.rebuild_with_eps(p, ep)), om, w, B, C, eta)
        Jm = oadj.objective_dense(osolve.dense_hbar(oadj.rebuild_with_eps(p, em)), om, w, B, C, eta)
        fd = (Jp - Jm) / (2 * h)
        # central differences: truncation h^2 |J'''| / 6 and rounding ~1e-16 |J| / h, both far
        # below 1e-6 of the derivative here
        assert abs(fd - g[r]) < 1e-6 * abs(fd), (r, fd, g[r])
    # and D_r is exactly dH/deps_r
    ep = p.eps.copy()
    ep[1] += 1.0
    dH = osolve.dense_hbar(oadj.rebuild_with_eps(p, ep)) - H
    assert np.abs(dH - np.diag(oadj.d_eps_diagonal(o, v, 1))).max() < 1e-12


def test_gradient_from_solutions_matches_finite_differences(model):
    """The gradient assembled from forward and adjoint solutions (the form the full-size check
    uses, with X and Y from any solver) against central finite differences of J, and against
    the dense-solve gradient."""
    p, hb, H, lam, ps, B, C = model
    o, v = p.o, p.v
    eta = 0.02
    om = np.linspace(-lam[0] - 0.2, -lam[0] + 0.2, 7)
    w = oadj.trapezoid_weights(om)
    X = osolve.dense_solve(H, om, B, eta)                        # [nw, np, D]
    Y = osolve.dense_solve(H.T.copy(), om, C.T.copy(), eta)      # adjoint: M^T y_p = c_p
    g = oadj.gradient_from_solutions(X, Y, w, o, v)
    assert np.abs(g - oadj.gradient_dense(H, om, w, B, C, eta, o, v)).max() <= 1e-12 * np.abs(g).max()
    h = 1e-5
    for r in (0, 2, o - 1, o, o + v - 1):
        ep, em = p.eps.copy(), p.eps.copy()
        ep[r] += h
        em[r] -= h
        Jp = oadj.objective_dense(osolve.dense_hbar(oadj.rebuild_with_eps(p, ep)), om, w, B, C, eta)
        Jm = oadj.objective_dense(osolve.dense_hbar(oadj.rebuild_with_eps(p, em)), om, w, B, C, eta)
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g[r]) < 1e-6 * abs(fd), (r, fd, g[r])
    # one-hot weights pick single frequencies: the sum over frequencies is linear in w
    g2 = sum(oadj.gradient_from_solutions(X[k:k + 1], Y[k:k + 1], w[k:k + 1], o, v)
             for k in range(len(om)))
    assert np.abs(g2 - g).max() <= 1e-13 * np.abs(g).max()


def test_orth_append_deflation():
    """Deflation of the basis (Eq. model's orthonormal S): dependent columns are dropped and
    independent ones kept, with the threshold relative to each column's own norm."""
    rng = np.random.default_rng(11)
    D, tol = 40, 1e-10
    S = omor.orth_append(np.zeros((D, 0)), rng.standard_normal((D, 5)), tol)
    assert S.shape == (D, 5)
    assert np.abs(S.T @ S - np.eye(5)).max() < 1e-14
    # a copy of a column of S, and a combination of its columns, add nothing
    assert omor.orth_append(S, S[:, 2:3] * 3.0, tol).shape[1] == 5
    comb = S @ rng.standard_normal(5)
    assert omor.orth_append(S, comb[:, None], tol).shape[1] == 5
    # two dependent columns in one call: the second is dropped against the first
    new = rng.standard_normal(D)
    T = omor.orth_append(S, np.stack([new, 2.0 * new + S[:, 0]], 1), tol)
    assert T.shape[1] == 6
    # the zero column is dropped
    assert omor.orth_append(S, np.zeros((D, 1)), tol).shape[1] == 5
    # a remainder of 1e3 tol relative to the column is kept; 1e-3 tol is dropped
    u = rng.standard_normal(D)
    u -= S @ (S.T @ u)
    u -= S @ (S.T @ u)
    u /= np.linalg.norm(u)
    # (at column scales 1e-6 .. 1e6, so that an absolute threshold would fail)
    for scale in (1e-6, 1.0, 1e6):
        for rel, kept in ((1e3 * tol, True), (1e-3 * tol, False)):
            col = scale * (comb + rel * np.linalg.norm(comb) * u)
            T = omor.orth_append(S, col[:, None], tol)
            assert T.shape[1] == (6 if kept else 5), (scale, rel)
            if kept:
                assert abs(abs(T[:, 5] @ u) - 1.0) < 1e-6
                assert np.abs(T.T @ T - np.eye(6)).max() < 1e-12


def test_rom_reextension_at_sampled_frequencies_adds_nothing(model):
    """Solving again at frequencies already in S gives columns inside span S: the order stays
    the same and the model is unchanged."""
    p, hb, H, lam, ps, B, C = model
    eta = 0.01
    wk = np.linspace(-lam[0] - 0.3, -lam[0] + 0.3, 3)
    rom = omor.ROM(hb, ps, eta, C, omor.dense_solver(H, B, eta))
    rom.extend(wk, 1e-10)
    m0 = rom.m
    om = np.linspace(wk[0], wk[-1], 9)
    G0, _ = rom.eval(om)
    rom.extend(wk[1:2], 1e-10)
    assert rom.m == m0
    G1, _ = rom.eval(om)
    assert np.abs(G1 - G0).max() < 1e-12 * np.abs(G0).max()
