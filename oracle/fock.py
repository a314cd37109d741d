"""Brute-force Fock-space construction of the IP-GFCC operator (tiny models only).

Nothing here uses a diagrammatic formula. Operators are explicit matrices between fixed
particle-number sectors of n = o + v spin orbitals:

* H = sum_pq h_pq a+_p a_q + 1/4 sum_pqrs <pq||rs> a+_p a+_q a_s a_r, with
  h_pq = f_pq - sum_i <pi||qi> so that the Fock matrix of the reference |Phi> (orbitals
  0..o-1 occupied) is f = diag(eps);
* T = sum t_i^a a+_a a_i + 1/4 sum t_ij^ab a+_a a+_b a_j a_i and Lambda likewise with the
  de-excitation strings; e^{+-T} by its (terminating) power series;
* H-bar = e^{-T} H e^{T} (the similarity transform of the paper's Methodology section);
* the IP space is spanned by |Phi_i> = a_i|Phi> and |Phi_ij^a> = a+_a a_j a_i|Phi> (i<j), the
  one-hole and two-hole-one-particle parts of X_p (the paper's auxiliary operator, Eq. xp);
* the IP matrix is the connected (commutator) part <Phi_mu| [H-bar, R_nu] |Phi>, the reading
  of "normal-product H-bar_N = H-bar - E_0" used throughout this repository;
* b_p = P_IP e^{-T} a_p e^{T} |Phi> (right-hand side of Eq. xplin);
* c_q,mu = <Phi|(1+Lambda) e^{-T} a+_q e^{T}|Phi_mu> (the rows c^T of Eq. gfcclineqn).

This is test infrastructure: it is the trust anchor that the closed forms are checked against.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np


def _popcount_below(det: int, p: int) -> int:
    return bin(det & ((1 << p) - 1)).count("1")


@lru_cache(maxsize=None)
def sector(n: int, nel: int):
    """Determinants (bitmasks) with nel electrons in n orbitals, and their index map."""
    dets = []
    for occ in itertools.combinations(range(n), nel):
        d = 0
        for p in occ:
            d |= 1 << p
        dets.append(d)
    dets.sort()
    return tuple(dets), {d: k for k, d in enumerate(dets)}


def annihilator(n: int, nel: int, p: int) -> np.ndarray:
    """Matrix of a_p from the nel sector to the nel-1 sector."""
    src, _ = sector(n, nel)
    _, dst_idx = sector(n, nel - 1)
    m = np.zeros((len(dst_idx), len(src)))
    for k, d in enumerate(src):
        if d >> p & 1:
            sign = -1.0 if _popcount_below(d, p) % 2 else 1.0
            m[dst_idx[d & ~(1 << p)], k] = sign
    return m


def creator(n: int, nel: int, p: int) -> np.ndarray:
    """Matrix of a+_p from the nel sector to the nel+1 sector."""
    return annihilator(n, nel + 1, p).T.copy()


class Ops:
    """Single-operator matrices for the sectors needed (nel, nel-1 and their pair sectors)."""

    def __init__(self, n: int):
        self.n = n
        self._a = {}

    def a(self, nel, p):
        key = ("a", nel, p)
        if key not in self._a:
            self._a[key] = annihilator(self.n, nel, p)
        return self._a[key]

    def c(self, nel, p):
        key = ("c", nel, p)
        if key not in self._a:
            self._a[key] = creator(self.n, nel, p)
        return self._a[key]


def hamiltonian(ops: Ops, nel: int, h: np.ndarray, eri: np.ndarray) -> np.ndarray:
    n = ops.n
    dim = len(sector(n, nel)[0])
    H = np.zeros((dim, dim))
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0.0 and nel >= 1:
                H += h[p, q] * (ops.c(nel - 1, p) @ ops.a(nel, q))
    if nel >= 2:
        # pair operators a_s a_r (nel -> nel-2) and a+_p a+_q (nel-2 -> nel)
        for r in range(n):
            for s in range(n):
                if r == s:
                    continue
                ann = ops.a(nel - 1, s) @ ops.a(nel, r)
                coef = eri[:, :, r, s]
                if not np.any(coef):
                    continue
                for p in range(n):
                    for q in range(n):
                        if p == q or coef[p, q] == 0.0:
                            continue
                        H += 0.25 * coef[p, q] * (ops.c(nel - 1, p) @ ops.c(nel - 2, q) @ ann)
    return H


def cluster(ops: Ops, nel: int, o: int, t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """T = sum t_i^a a+_a a_i + 1/4 sum t_ij^ab a+_a a+_b a_j a_i in the nel sector."""
    n = ops.n
    dim = len(sector(n, nel)[0])
    T = np.zeros((dim, dim))
    v = n - o
    for i in range(o):
        for a in range(v):
            if nel >= 1:
                T += t1[i, a] * (ops.c(nel - 1, o + a) @ ops.a(nel, i))
    if nel >= 2:
        for i in range(o):
            for j in range(o):
                if i == j:
                    continue
                ann = ops.a(nel - 1, j) @ ops.a(nel, i)
                for a in range(v):
                    for b in range(v):
                        if a == b:
                            continue
                        T += 0.25 * t2[i, j, a, b] * (ops.c(nel - 1, o + a) @ ops.c(nel - 2, o + b) @ ann)
    return T


def expm_nilpotent(T: np.ndarray, sign: float = 1.0) -> np.ndarray:
    out = np.eye(T.shape[0])
    term = np.eye(T.shape[0])
    for k in range(1, T.shape[0] + 2):
        term = term @ (sign * T) / k
        if not np.any(term):
            break
        out = out + term
    return out


class BruteForce:
    """All IP-GFCC objects of a tiny model, by explicit Fock-space matrices."""

    def __init__(self, o, v, eps, t1, t2, eri, l1=None, l2=None):
        self.o, self.v, self.n = o, v, o + v
        n = self.n
        f = np.diag(eps)
        h = f - np.einsum("piqi->pq", eri[:, :o, :, :o])
        self.ops = ops = Ops(n)
        self.H0 = hamiltonian(ops, o, h, eri)
        self.H1 = hamiltonian(ops, o - 1, h, eri)
        T0 = cluster(ops, o, o, t1, t2)
        T1m = cluster(ops, o - 1, o, t1, t2)
        self.eT0, self.emT0 = expm_nilpotent(T0, 1.0), expm_nilpotent(T0, -1.0)
        self.eT1, self.emT1 = expm_nilpotent(T1m, 1.0), expm_nilpotent(T1m, -1.0)
        self.Hb0 = self.emT0 @ self.H0 @ self.eT0
        self.Hb1 = self.emT1 @ self.H1 @ self.eT1
        l1 = t1 if l1 is None else l1
        l2 = t2 if l2 is None else l2
        # Lambda^dagger has the excitation form, so <Phi|(1+Lambda) = ((1+Lambda^dagger)|Phi>)^T
        self.Ldag0 = cluster(ops, o, o, l1, l2)
        dets0, idx0 = sector(n, o)
        self.phi = np.zeros(len(dets0))
        self.phi[idx0[(1 << o) - 1]] = 1.0
        # IP basis: R_nu operators (nel=o -> o-1) and the states R_nu|Phi>
        self.R = []
        for i in range(o):
            self.R.append(ops.a(o, i))
        for i in range(o):
            for j in range(i + 1, o):
                ann = ops.a(o - 1, j) @ ops.a(o, i)
                for a in range(v):
                    self.R.append(ops.c(o - 2, o + a) @ ann)
        self.basis = np.stack([R @ self.phi for R in self.R], axis=1)  # (dim_{o-1}, D)
        self.D = self.basis.shape[1]

    def ip_matrix(self) -> np.ndarray:
        """sigma_mu,nu = <Phi_mu| [H-bar, R_nu] |Phi>."""
        B = self.basis
        hphi = self.Hb0 @ self.phi
        cols = []
        for R, st in zip(self.R, B.T):
            cols.append(B.T @ (self.Hb1 @ st - R @ hphi))
        return np.stack(cols, axis=1)

    def ip_matrix_full(self) -> np.ndarray:
        """<Phi_mu| H-bar |Phi_nu> (no commutator) -- for the E_0 / residual bookkeeping test."""
        B = self.basis
        return B.T @ self.Hb1 @ B

    def e_cc(self) -> float:
        return float(self.phi @ self.Hb0 @ self.phi)

    def b(self, p: int) -> np.ndarray:
        """P_IP e^{-T} a_p e^{T}|Phi>."""
        st = self.emT1 @ self.ops.a(self.o, p) @ self.eT0 @ self.phi
        return self.basis.T @ st

    def c(self, q: int) -> np.ndarray:
        """c_q,mu = <Phi|(1+Lambda) e^{-T} a+_q e^{T} |Phi_mu>."""
        bra = (self.phi + self.Ldag0 @ self.phi) @ self.emT0 @ self.ops.c(self.o - 1, q) @ self.eT1
        return bra @ self.basis
