"""Shifted linear solves, Green's function and spectral function (the plain GFCC path).

Eq. xplin asks for X_p(omega) with (omega - i eta + H-bar_N) X_p = b_p for each orbital p and
frequency omega; Eq. gfcclineqn gives G(omega) = c^T X(omega) (plain transpose, no complex
conjugation) and the spectral function follows from the imaginary part of the diagonal of G.

Sign reading: with the paper's operator (omega - i eta + H-bar_N) and H-bar_N's 1h diagonal
equal to -eps_i, the non-interacting limit is G_ii = 1/(omega - eps_i - i eta), whose
imaginary part is positive. A(omega) is reported as +(1/pi) sum_p Im G_pp(omega) >= 0, the
positive peak curve that the paper plots.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import sigma as sg


def dense_hbar(hb) -> np.ndarray:
    """H-bar_N as a dense D x D matrix, one column per unit vector through the sigma product."""
    D = sg.dim(hb.o, hb.v)
    return sg.sigma(hb, np.eye(D)).T.copy()


def shifted(H: np.ndarray, omega: float, eta: float) -> np.ndarray:
    return H + (omega - 1j * eta) * np.eye(H.shape[0])


def dense_solve(H: np.ndarray, omegas, B: np.ndarray, eta: float) -> np.ndarray:
    """X[w] = ((omega_w - i eta) I + H)^{-1} B  by LU; B is D x np; returns [nw, np, D]."""
    out = np.empty((len(omegas), B.shape[1], H.shape[0]), dtype=np.complex128)
    for w, om in enumerate(omegas):
        out[w] = sla.solve(shifted(H, om, eta), B.astype(np.complex128)).T
    return out


def green(C: np.ndarray, X: np.ndarray) -> np.ndarray:
    """G[w, q, p] = c_q^T X_p(omega_w); C is [nq, D], X is [nw, np, D]."""
    return np.einsum("qd,wpd->wqp", C, X)


def spectral(G: np.ndarray) -> np.ndarray:
    """A(omega) = (1/pi) sum_p Im G_pp(omega) for G[w, p, p]."""
    return np.einsum("wpp->w", G.imag) / np.pi


def sum_over_states(H: np.ndarray, omegas, B, C, eta) -> np.ndarray:
    """G from the eigen-decomposition H = R diag(lam) R^{-1} (the Introduction's route):
    G_qp(omega) = sum_k (c_q^T r_k)(l_k^T b_p) / (omega - i eta + lam_k)."""
    lam, R = np.linalg.eig(H)
    Linv = np.linalg.inv(R)
    left = C @ R          # [nq, K]
    right = Linv @ B      # [K, np]
    den = (np.asarray(omegas)[:, None] - 1j * eta) + lam[None, :]
    return np.einsum("qk,kp,wk->wqp", left, right, 1.0 / den)


class Operator:
    """Matrix-free M(omega) = (omega - i eta) I + H-bar_N through the closed-form sigma."""

    def __init__(self, hb, transpose: bool = False):
        self.hb = hb
        self.D = sg.dim(hb.o, hb.v)
        self.diag = sg.diagonal(hb)
        self.transpose = transpose
        self.nmatvec = 0

    def hbar(self, x):
        self.nmatvec += 1
        return sg.sigma_t(self.hb, x) if self.transpose else sg.sigma(self.hb, x)


def gmres(op: Operator, b: np.ndarray, omega: float, eta: float, tol: float = 1e-10,
          restart: int = 50, maxit: int = 5000, x0=None):
    """Right-preconditioned restarted GMRES for M(omega) x = b.

    Preconditioner P = diag(M(omega)) (Jacobi), applied on the right so the minimised
    residual is the true residual. Arnoldi uses classical Gram-Schmidt with one full
    re-orthogonalisation pass (CGS2). Stops when the true relative residual
    ||b - M x|| / ||b|| <= tol, recomputed explicitly at each restart.
    Returns (x, iterations, relative residual).
    """
    shift = omega - 1j * eta
    pdiag = op.diag + shift
    bnorm = np.linalg.norm(b)
    x = np.zeros(op.D, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    if bnorm == 0.0:
        return np.zeros(op.D, dtype=np.complex128), 0, 0.0

    def M(z):
        return op.hbar(z) + shift * z

    it = 0
    r = b - M(x)
    rel = np.linalg.norm(r) / bnorm
    while rel > tol and it < maxit:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, op.D), dtype=np.complex128)
        Hm = np.zeros((restart + 1, restart), dtype=np.complex128)
        V[0] = r / beta
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        k_used = 0
        for k in range(restart):
            w = M(V[k] / pdiag)
            h = np.zeros(k + 1, dtype=np.complex128)
            for _ in range(2):                      # CGS2
                hk = V[: k + 1].conj() @ w
                w = w - V[: k + 1].T @ hk
                h += hk
            hn = np.linalg.norm(w)
            Hm[: k + 1, k] = h
            Hm[k + 1, k] = hn
            # apply previous Givens rotations
            for j in range(k):
                t = cs[j].conj() * Hm[j, k] + sn[j].conj() * Hm[j + 1, k]
                Hm[j + 1, k] = -sn[j] * Hm[j, k] + cs[j] * Hm[j + 1, k]
                Hm[j, k] = t
            den = np.hypot(abs(Hm[k, k]), abs(Hm[k + 1, k]))
            cs[k] = Hm[k, k] / den
            sn[k] = Hm[k + 1, k] / den
            Hm[k, k] = den
            Hm[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k].conj() * g[k]
            it += 1
            k_used = k + 1
            if hn == 0.0:
                break
            V[k + 1] = w / hn
            if abs(g[k + 1]) / bnorm <= tol * 0.5 or it >= maxit:
                break
        y = sla.solve_triangular(Hm[:k_used, :k_used], g[:k_used])
        x = x + (V[:k_used].T @ y) / pdiag
        r = b - M(x)
        rel = np.linalg.norm(r) / bnorm
    return x, it, rel


def solve_points(hb, omegas, ps, eta, tol=1e-10, restart=50, maxit=5000, transpose=False,
                 rhs=None):
    """GMRES at every (omega, p). Returns X [nw, np, D], iterations and residuals [nw, np]."""
    op = Operator(hb, transpose=transpose)
    nw, npp = len(omegas), len(ps)
    X = np.empty((nw, npp, op.D), dtype=np.complex128)
    its = np.zeros((nw, npp), dtype=np.int64)
    res = np.zeros((nw, npp))
    for w, om in enumerate(omegas):
        for k, p in enumerate(ps):
            b = sg.b_vector(hb.o, hb.v, p) if rhs is None else rhs[k]
            X[w, k], its[w, k], res[w, k] = gmres(op, b, om, eta, tol, restart, maxit)
    return X, its, res
