"""Complex DIIS solver for the shifted GFCC systems -- TEST INFRASTRUCTURE ONLY.

The paper solves Eq. xplin with direct inversion in the iterative subspace (DIIS) carried
over to complex vectors, keeping 10 micro-iteration iterates (Results, the convergence study
of Fig. 3). It names the method and the subspace size and nothing else; the reading taken
here is the periodic DIIS of coupled-cluster codes:

* a micro-iteration is one Jacobi step x <- x + e with e = P^{-1} (b - M(omega) x),
  P = diag(M(omega)), M(omega) = (omega - i eta) I + H-bar_N; the pair (x after the step, e)
  is kept;
* after ndiis micro-iterations the kept iterates are combined, x <- sum_k c_k x_k, with the
  complex coefficients that minimise ||sum_k c_k e_k|| subject to sum_k c_k = 1; then the
  subspace starts afresh. The minimum is taken in its unconstrained form: with
  gamma_k = sum_{j<=k} c_j, sum_k c_k e_k = e_last - sum_k gamma_k (e_{k+1} - e_k), a linear
  least-squares problem over the differences of consecutive error vectors, solved by a
  library least-squares routine. (Pulay's bordered system over B_ij = e_i^H e_j states the
  same minimum, but forming B squares the condition number of the error vectors, which
  become nearly parallel as the iteration settles: cond(B) reaches 1e17 on small GFCC
  systems, where rounding alone then decides the combination);
* the stopping test is the true relative residual ||b - M x|| / ||b|| <= tol, evaluated before
  every micro-iteration; it also ends a column at maxit micro-iterations or at a non-finite
  residual.

Returns the relative residual of every evaluated iterate, the convergence profile that the
paper plots.
"""
from __future__ import annotations

import numpy as np

from . import sigma as sg
from . import solve as so


def extrapolate(xs, es):
    """sum_k c_k x_k with c minimising ||sum_k c_k e_k|| under sum_k c_k = 1, written as
    x_last - sum_k gamma_k (x_{k+1} - x_k) with gamma = argmin ||e_last - F gamma||,
    F = [e_{k+1} - e_k]."""
    m = len(es)
    if m == 1:
        return xs[0]
    F = np.stack([es[k + 1] - es[k] for k in range(m - 1)], 1)
    g, *_ = np.linalg.lstsq(F, es[-1], rcond=None)
    return xs[-1] - sum(g[k] * (xs[k + 1] - xs[k]) for k in range(m - 1))


def diis(op: so.Operator, b: np.ndarray, omega: float, eta: float, tol: float = 1e-10,
         ndiis: int = 10, maxit: int = 500, x0=None):
    """Periodic complex DIIS on M(omega) x = b. Returns (x, micro-iterations, relative
    residual, residual history)."""
    shift = omega - 1j * eta
    pdiag = op.diag + shift
    bnorm = np.linalg.norm(b)
    x = np.zeros(op.D, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    if bnorm == 0.0:
        return np.zeros(op.D, dtype=np.complex128), 0, 0.0, [0.0]
    hist = []
    it = 0
    while True:
        xs, es = [], []
        for _ in range(ndiis):
            r = b - (op.hbar(x) + shift * x)
            rel = np.linalg.norm(r) / bnorm
            hist.append(rel)
            if rel <= tol or it >= maxit or not np.isfinite(rel):
                return x, it, rel, hist
            e = r / pdiag
            x = x + e
            xs.append(x)
            es.append(e)
            it += 1
        x = extrapolate(xs, es)


def solve_points(hb, omegas, ps, eta, tol=1e-10, ndiis=10, maxit=500, transpose=False, rhs=None,
                 x0=None):
    """DIIS at every (omega, p). Returns X [nw, np, D], iterations and residuals [nw, np] and
    the histories (list of lists, index w * np + k). rhs: optional right-hand sides [np, D]
    (default b_p); x0: optional guesses [nw, np, D]."""
    op = so.Operator(hb, transpose=transpose)
    nw, npp = len(omegas), len(ps)
    X = np.empty((nw, npp, op.D), dtype=np.complex128)
    its = np.zeros((nw, npp), dtype=np.int64)
    res = np.zeros((nw, npp))
    hists = []
    for w, om in enumerate(omegas):
        for k, p in enumerate(ps):
            b = sg.b_vector(hb.o, hb.v, p) if rhs is None else rhs[k]
            g = None if x0 is None else x0[w, k]
            X[w, k], its[w, k], res[w, k], h = diis(op, b, om, eta, tol, ndiis, maxit, g)
            hists.append(h)
    return X, its, res, hists
