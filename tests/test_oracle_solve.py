"""Pins of the oracle's solve layer: dense LU, GMRES, sum over states, closed forms, moments."""
import numpy as np
import pytest

import synth
from oracle import hbar as ohbar
from oracle import sigma as osig
from oracle import solve as osolve


@pytest.fixture(scope="module")
def small():
    o, v = 6, 8
    p = synth.make_problem(o, v, 21)
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    ps = np.arange(o)
    B = np.stack([osig.b_vector(o, v, q) for q in ps], 1)
    C = np.stack([osig.c_vector(o, v, p.t1, p.t2, p.l1, p.l2, q) for q in ps], 0)
    return p, hb, H, ps, B, C


def test_noninteracting_green_function():
    """T = 0, V = 0: G_ii(omega) = 1/(omega - eps_i - i eta) exactly; A is a sum of Lorentzians."""
    o, v = 4, 5
    p = synth.make_problem(o, v, 2)
    z = np.zeros
    hb = ohbar.build_hbar(o, v, p.eps, z((o, v)), z((o, o, v, v)), z((o,) * 4), z((o, o, o, v)),
                          z((o, o, v, v)), z((o, v, v, o)), z((o, v, v, v)))
    H = osolve.dense_hbar(hb)
    om = np.linspace(-1.6, -0.2, 31)
    eta = 0.01
    B = np.stack([osig.b_vector(o, v, q) for q in range(o)], 1)
    C = np.stack([osig.c_vector(o, v, z((o, v)), z((o, o, v, v)), z((o, v)), z((o, o, v, v)), q)
                  for q in range(o)], 0)
    G = osolve.green(C, osolve.dense_solve(H, om, B, eta))
    ref = 1.0 / (om[:, None] - p.eps[None, :o] - 1j * eta)
    assert np.abs(np.einsum("wii->wi", G) - ref).max() < 1e-12
    A = osolve.spectral(G)
    lor = (eta / np.pi) / ((om[:, None] - p.eps[None, :o]) ** 2 + eta ** 2)
    assert np.abs(A - lor.sum(1)).max() < 1e-10


def test_gmres_matches_dense(small):
    p, hb, H, ps, B, C = small
    om = np.array([-1.4, -0.9, -0.35])
    Xd = osolve.dense_solve(H, om, B, 0.01)
    X, its, res = osolve.solve_points(hb, om, ps, 0.01, tol=1e-12, restart=20)
    assert res.max() <= 1e-12
    assert np.abs(X - Xd).max() < 1e-10 * np.abs(Xd).max()


def test_sum_over_states(small):
    """G from the eigen-decomposition of H-bar equals G from the shifted solves."""
    p, hb, H, ps, B, C = small
    om = np.linspace(-2.0, -0.3, 17)
    G1 = osolve.green(C, osolve.dense_solve(H, om, B, 0.02))
    G2 = osolve.sum_over_states(H, om, B, C, 0.02)
    assert np.abs(G1 - G2).max() < 1e-9 * np.abs(G1).max()


def test_high_frequency_moments(small):
    """Large |omega|: G = c.b/z - c^T H b/z^2 + ..., z = omega - i eta, so
    omega G_pp -> c_p.b_p and omega (omega G - c.b) -> -c^T (H - i eta) b, with remainders
    bounded by the next moment over |omega|."""
    p, hb, H, ps, B, C = small
    eta = 0.01
    Hs = H - 1j * eta * np.eye(H.shape[0])
    m0 = np.diag(C @ B)
    m1 = -np.diag(C @ Hs @ B)
    m2 = np.diag(C @ Hs @ Hs @ B)
    for om in (-1e4, 1e4, -1e5):
        G = osolve.green(C, osolve.dense_solve(H, [om], B, eta))[0]
        first = om * np.diag(G)
        assert np.all(np.abs(first - m0) <= 2 * (np.abs(m1) + 1e-3) / abs(om))
        second = om * (first - m0)
        assert np.all(np.abs(second - m1) <= 2 * (np.abs(m2) + 1e-3) / abs(om) + 1e-6)


def test_bj_sign_convention_is_complex_conjugate(small):
    """(omega - H' + i eta) X' = b with H' = -H-bar_N gives X' = conj(X)."""
    p, hb, H, ps, B, C = small
    om, eta = -0.8, 0.01
    X = np.linalg.solve(osolve.shifted(H, om, eta), B.astype(complex))
    Xp = np.linalg.solve(om * np.eye(H.shape[0]) + H + 1j * eta * np.eye(H.shape[0]), B.astype(complex))
    assert np.abs(Xp - X.conj()).max() < 1e-13


def test_o10v20_spectrum_report():
    """Small case (o=10, v=20): dense eigenvalues of H-bar_N are real-dominated (max |Im| < eta) and lie above
    the frequency window, so A(omega) > 0 on it."""
    cfg = synth.WORKLOADS["o10v20"]
    p = synth.make_problem(cfg["o"], cfg["v"], cfg["seed"])
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    lam = np.linalg.eigvals(H)
    assert np.abs(lam.imag).max() < cfg["eta"]
    assert lam.real.min() > 1.0
    om = synth.omega_grid(cfg["omega"])
    ps = synth.valence_p(cfg["o"], cfg["np"])
    B = np.stack([osig.b_vector(p.o, p.v, q) for q in ps], 1)
    C = np.stack([osig.c_vector(p.o, p.v, p.t1, p.t2, p.l1, p.l2, q) for q in ps], 0)
    A = osolve.spectral(osolve.green(C, osolve.dense_solve(H, om[::8], B, cfg["eta"])))
    assert np.all(A > 0)
