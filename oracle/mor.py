"""Reduced-order model of the GFCC linear system (Methodology: Eq. model and the adaptive
refinement described after it). Test infrastructure only.

Steps, in the paper's order:
1. solve the full system at sampled frequencies omega_k;
2. orthonormalise the auxiliary vectors X_p(omega_k) into S (here: the real and imaginary
   parts, so that S is real and S^T = S^H -- the reading that keeps <v_i|v_j> = delta_ij
   together with S^T in the projection);
3. project: Hhat = S^T H S, bhat = S^T b, chat^T = c^T S;
4. solve the small shifted systems on the dense grid;
5. estimate the error between adjacent sampled frequencies and add midpoints until the
   largest estimate is below the threshold or the order bound is reached.
The error estimate is the relative full-space residual of the reduced solution, computed
here explicitly as ||b - (omega - i eta) S xhat - H S xhat|| / ||b||.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import sigma as sg
from . import solve as so


def orth_append(S: np.ndarray, cols: np.ndarray, defl_tol: float) -> np.ndarray:
    """Append columns to the orthonormal S (D x m) by classical Gram-Schmidt applied twice per
    column; a column whose norm falls below defl_tol times its original norm is dropped."""
    out = [S[:, i] for i in range(S.shape[1])]
    for c in cols.T:
        w = c.copy()
        n0 = np.linalg.norm(w)
        if n0 == 0.0:
            continue
        for _ in range(2):
            if out:
                Q = np.stack(out, 1)
                w = w - Q @ (Q.T @ w)
        n1 = np.linalg.norm(w)
        if n1 > defl_tol * n0:
            out.append(w / n1)
    return np.stack(out, 1) if out else np.zeros((S.shape[0], 0))


class ROM:
    def __init__(self, hb, ps, eta, C, solver):
        self.hb, self.ps, self.eta = hb, np.asarray(ps), eta
        self.D = sg.dim(hb.o, hb.v)
        self.S = np.zeros((self.D, 0))
        self.HS = np.zeros((self.D, 0))
        self.C = C                  # [np, D] c_q rows
        self.B = np.stack([sg.b_vector(hb.o, hb.v, p) for p in ps], 1)  # [D, np]
        self.omega_k: list[float] = []
        self.solver = solver        # (omegas) -> X [nw, np, D]

    def extend(self, omegas, defl_tol):
        X = self.solver(np.asarray(omegas))
        cols = []
        for w in range(X.shape[0]):
            for k in range(X.shape[1]):
                cols.append(X[w, k].real)
                cols.append(X[w, k].imag)
        m0 = self.S.shape[1]
        self.S = orth_append(self.S, np.stack(cols, 1), defl_tol)
        new = self.S[:, m0:]
        if new.shape[1]:
            self.HS = np.concatenate([self.HS, sg.sigma(self.hb, new.T).T], 1)
        self.omega_k += list(omegas)

    @property
    def m(self):
        return self.S.shape[1]

    def projected(self):
        Hhat = self.S.T @ self.HS
        bhat = self.S.T @ self.B
        chat = self.C @ self.S
        return Hhat, bhat, chat

    def eval(self, omegas):
        """Ghat [nw, nq, np] and the max-over-p relative residual [nw]."""
        Hhat, bhat, chat = self.projected()
        G = np.empty((len(omegas), len(self.ps), len(self.ps)), dtype=complex)
        res = np.empty(len(omegas))
        bn = np.linalg.norm(self.B, axis=0)
        for w, om in enumerate(omegas):
            z = om - 1j * self.eta
            xh = sla.solve(Hhat + z * np.eye(self.m), bhat.astype(complex))
            G[w] = chat @ xh
            R = self.B - z * (self.S @ xh) - self.HS @ xh
            res[w] = np.max(np.linalg.norm(R, axis=0) / bn)
        return G, res


def lift(rom: ROM, omegas) -> np.ndarray:
    """Full-space approximate solutions S xhat_p(omega) [nw, np, D] of the reduced model: the
    initial guesses for full solves that the reduced model provides (the model's by-product
    described with Eq. model)."""
    Hhat, bhat, _ = rom.projected()
    X = np.empty((len(omegas), len(rom.ps), rom.D), dtype=complex)
    for w, om in enumerate(omegas):
        z = om - 1j * rom.eta
        xh = sla.solve(Hhat + z * np.eye(rom.m), bhat.astype(complex))   # [m, np]
        X[w] = (rom.S @ xh).T
    return X


def refine(rom: ROM, grid, wmin, wmax, per_round, resid_tol, max_order, max_rounds, defl_tol):
    """Midpoint refinement; returns (rounds, final max residual on the window's grid)."""
    g = np.sort(np.asarray([w for w in grid if wmin <= w <= wmax]))
    rounds = 0
    while True:
        _, res = rom.eval(g)
        rmax = res.max()
        if rmax <= resid_tol or rounds >= max_rounds or rom.m >= max_order:
            return rounds, rmax
        ks = np.unique(np.concatenate([rom.omega_k, [wmin, wmax]]))
        iv = []
        for lo, hi in zip(ks[:-1], ks[1:]):
            if hi < wmin or lo > wmax:
                continue
            inside = (g >= lo) & (g <= hi)
            e = res[inside].max() if inside.any() else 0.0
            if e > resid_tol:
                iv.append((-e, lo, hi))
        if not iv:
            return rounds, rmax
        iv.sort()  # largest error first, ties toward lower omega
        add = [0.5 * (lo + hi) for (_, lo, hi) in iv[:per_round]]
        rom.extend(add, defl_tol)
        rounds += 1


def dense_solver(H, B, eta):
    def f(omegas):
        return so.dense_solve(H, omegas, B, eta)
    return f
