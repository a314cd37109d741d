"""Pins of the oracle's complex DIIS solver against facts it does not compute itself: the
equivalence of one DIIS cycle with a minimal-residual Krylov solve, the Neumann series of the
plain Jacobi iteration, the diagonal limit and the dense LU solution."""
import numpy as np
import pytest

import synth
from oracle import diis as odiis
from oracle import hbar as ohbar
from oracle import sigma as osig
from oracle import solve as osolve


class DenseOp:
    """A dense complex H with the interface of the matrix-free operator."""

    def __init__(self, H):
        self.H = H
        self.D = H.shape[0]
        self.diag = H.diagonal().copy()

    def hbar(self, x):
        return self.H @ x


def dense_problem(n, seed, offdiag=0.35):
    rng = np.random.default_rng(seed)
    H = offdiag * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    H += np.diag(rng.uniform(-2.0, 2.0, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x0 = 0.1 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    return DenseOp(H), b, x0


@pytest.mark.parametrize("m", [2, 4, 7])
def test_one_cycle_is_krylov_minimal_residual_then_jacobi(m):
    """For a linear system, the preconditioned residual is affine in x, so the DIIS combination
    of the iterates x_0 .. x_{m-1} (whose residuals are the kept e_k) is the point y of
    x_0 + K_{m-1}(P^-1 M, z_0) with the least preconditioned residual, z_0 = P^-1 (b - M x_0);
    the kept pairs (x_{k+1}, e_k) then return one Jacobi step from y. Here y comes from a
    least-squares solve on an explicit Krylov basis."""
    op, b, x0 = dense_problem(30, 5 + m)
    omega, eta = 0.3, 0.05
    shift = omega - 1j * eta
    M = op.H + shift * np.eye(op.D)
    P = op.diag + shift
    A = M / P[:, None]
    z0 = (b - M @ x0) / P
    K = [z0]
    for _ in range(m - 2):
        K.append(A @ K[-1])
    K = np.stack(K, 1)
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(A @ Q, z0, rcond=None)
    y = x0 + Q @ c
    expect = y + (b - M @ y) / P
    x, it, rel, hist = odiis.diis(op, b, omega, eta, tol=1e-300, ndiis=m, maxit=m, x0=x0)
    assert it == m and len(hist) == m + 1
    assert np.abs(x - expect).max() <= 1e-10 * np.abs(expect).max()
    assert rel == pytest.approx(np.linalg.norm(b - M @ expect) / np.linalg.norm(b), rel=1e-8)


def test_single_iterate_is_the_jacobi_neumann_series():
    """ndiis = 1 keeps one iterate with coefficient 1: x_k = sum_{j<k} (I - P^-1 M)^j P^-1 b."""
    op, b, _ = dense_problem(25, 3, offdiag=0.2)
    omega, eta = -0.4, 0.02
    shift = omega - 1j * eta
    M = op.H + shift * np.eye(op.D)
    P = op.diag + shift
    T = np.eye(op.D) - M / P[:, None]
    k = 9
    expect = sum(np.linalg.matrix_power(T, j) @ (b / P) for j in range(k))
    x, it, rel, hist = odiis.diis(op, b, omega, eta, tol=1e-300, ndiis=1, maxit=k)
    assert it == k
    assert np.abs(x - expect).max() <= 1e-12 * np.abs(expect).max()


def test_exact_after_one_cycle_when_the_krylov_space_is_full():
    """With m - 1 >= n the Krylov space is the whole space: one cycle gives the solution."""
    op, b, _ = dense_problem(5, 11, offdiag=0.8)
    omega, eta = 0.1, 0.03
    M = op.H + (omega - 1j * eta) * np.eye(op.D)
    x, it, rel, hist = odiis.diis(op, b, omega, eta, tol=1e-13, ndiis=7, maxit=50)
    assert it == 7 and rel <= 1e-13
    assert np.abs(x - np.linalg.solve(M, b)).max() <= 1e-12 * np.abs(x).max()


def test_diagonal_operator_converges_in_one_step():
    """T = 0 and V = 0 make H-bar_N diagonal, so the Jacobi step is the exact inverse:
    x_1 = b / (omega - i eta - eps_p) and the next residual vanishes."""
    o, v = 4, 5
    p = synth.make_problem(o, v, 2)
    z = np.zeros
    hb = ohbar.build_hbar(o, v, p.eps, z((o, v)), z((o, o, v, v)), z((o,) * 4), z((o, o, o, v)),
                          z((o, o, v, v)), z((o, v, v, o)), z((o, v, v, v)))
    X, its, res, hists = odiis.solve_points(hb, [-0.7, -0.25], range(o), 0.01, tol=1e-14)
    assert np.all(its == 1) and res.max() <= 1e-15
    for w, om in enumerate([-0.7, -0.25]):
        for q in range(o):
            assert X[w, q, q] == pytest.approx(1.0 / (om - p.eps[q] - 0.01j), rel=1e-15)
            h = hists[w * o + q]
            assert len(h) == 2 and h[0] == 1.0 and h[1] <= 1e-15


def test_exact_guess_takes_no_iteration_and_zero_rhs():
    op, b, _ = dense_problem(12, 8)
    M = op.H + (0.2 - 0.01j) * np.eye(op.D)
    xs = np.linalg.solve(M, b)
    x, it, rel, hist = odiis.diis(op, b, 0.2, 0.01, tol=1e-12, x0=xs)
    assert it == 0 and rel <= 1e-12 and len(hist) == 1
    x, it, rel, hist = odiis.diis(op, np.zeros(12), 0.2, 0.01)
    assert it == 0 and rel == 0.0 and not x.any()


def test_gfcc_solutions_match_dense_lu():
    """On the GFCC operator the converged DIIS solutions equal the LU solutions; near the
    bottom of the window it needs more micro-iterations than GMRES needs Arnoldi steps."""
    o, v = 6, 8
    p = synth.make_problem(o, v, 1)
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    ps = [0, 3, 5]
    B = np.stack([osig.b_vector(o, v, q) for q in ps], 1)
    om = [-0.9, -0.5, -0.3]
    Xd = osolve.dense_solve(H, om, B, 0.01)
    X, its, res, hists = odiis.solve_points(hb, om, ps, 0.01, tol=1e-12, maxit=400)
    assert res.max() <= 1e-12
    assert np.abs(X - Xd).max() <= 1e-9 * np.abs(Xd).max()
    _, gits, _ = osolve.solve_points(hb, om, ps, 0.01, tol=1e-12, restart=30)
    assert its.sum() > gits.sum()


def test_transpose_systems_match_dense_lu():
    o, v = 5, 6
    p = synth.make_problem(o, v, 4)
    hb = ohbar.build_hbar_from_problem(p)
    H = osolve.dense_hbar(hb)
    C = np.stack([osig.c_vector(o, v, p.t1, p.t2, p.l1, p.l2, q) for q in range(o)], 0)
    om = [-0.45]
    X, its, res, _ = odiis.solve_points(hb, om, range(o), 0.01, tol=1e-12, maxit=400,
                                        transpose=True, rhs=C)
    Yd = osolve.dense_solve(H.T.copy(), om, C.T.copy(), 0.01)
    assert res.max() <= 1e-12
    assert np.abs(X - Yd).max() <= 1e-9 * np.abs(Yd).max()
