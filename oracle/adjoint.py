"""Gradient of windowed spectral weight with respect to orbital energies. Test infrastructure.

J = sum_k w_k A(omega_k), A = (1/pi) sum_p Im G_pp, G_pp = c_p^T M(omega)^{-1} b_p with
M(omega) = (omega - i eta) I + H-bar_N. With amplitudes held fixed, the orbital energies enter
H-bar_N only through the diagonal Fock blocks F_mi and F_ae, so dM/deps_r = D_r is diagonal in
the packed basis:
  occupied r:  -1 on the one-hole entry r and on every 2h1p entry (ij,a) with r in {i, j};
  virtual  r:  +1 on every 2h1p entry (ij,a) with a = r - o.
Then dG_pp/deps_r = -y_p^T D_r x_p with M^T y_p = c_p and M x_p = b_p.
"""
from __future__ import annotations

import numpy as np

from . import hbar as hbar_mod
from . import sigma as sg
from . import solve as so


def d_eps_diagonal(o: int, v: int, r: int) -> np.ndarray:
    D = sg.dim(o, v)
    d = np.zeros(D)
    iu, ju = sg.pair_index(o)
    two = np.zeros((len(iu), v))
    if r < o:
        d[r] = -1.0
        two[(iu == r) | (ju == r), :] = -1.0
    else:
        two[:, r - o] = 1.0
    d[o:] = two.reshape(-1)
    return d


def objective_dense(H, omegas, weights, B, C, eta) -> float:
    X = so.dense_solve(H, omegas, B, eta)
    A = so.spectral(so.green(C, X))
    return float(np.dot(weights, A))


def gradient_dense(H, omegas, weights, B, C, eta, o, v) -> np.ndarray:
    """dJ/deps_r for every orbital r (dense solves)."""
    grad = np.zeros(o + v)
    Dr = np.stack([d_eps_diagonal(o, v, r) for r in range(o + v)])  # [o+v, D]
    for w, om in enumerate(omegas):
        M = so.shifted(H, om, eta)
        X = np.linalg.solve(M, B.astype(complex))        # [D, np]
        Y = np.linalg.solve(M.T, C.T.astype(complex))    # [D, np]
        q = np.einsum("dp,dp->d", Y, X)                   # sum_p y_p * x_p elementwise
        grad += weights[w] * (-(Dr @ q)).imag / np.pi
    return grad


def gradient_from_solutions(X, Y, weights, o, v) -> np.ndarray:
    """Same formula from solutions X, Y [nw, np, D] (forward and adjoint)."""
    grad = np.zeros(o + v)
    Dr = np.stack([d_eps_diagonal(o, v, r) for r in range(o + v)])
    q = np.einsum("w,wpd,wpd->d", np.asarray(weights, dtype=complex), Y, X)
    return (-(Dr @ q)).imag / np.pi


def trapezoid_weights(omegas) -> np.ndarray:
    om = np.asarray(omegas)
    w = np.zeros(len(om))
    h = np.diff(om)
    w[:-1] += 0.5 * h
    w[1:] += 0.5 * h
    return w


def rebuild_with_eps(prob, eps):
    """H-bar with perturbed orbital energies and the original amplitudes (held fixed)."""
    return hbar_mod.build_hbar(prob.o, prob.v, eps, prob.t1, prob.t2, prob.block("oooo"),
                               prob.block("ooov"), prob.block("oovv"), prob.block("ovvo"),
                               prob.block("ovvv"))
