"""Seeded synthetic inputs for the IP-GFCC problem (orbital energies, amplitudes, integrals).

This module holds none of the Green's-function method: it draws the random inputs that both
the CPU oracle and the GPU path consume. Values are pure functions of (seed, stream, index),
produced by the counter-based generator in ``synth.c`` (SplitMix64 + Box-Muller).

Recipe (the paper's molecules are replaced by random spin-orbital models of the same shape):

* occupied energies  U[-1.5, -0.3] Ha, virtual energies U[0.1, 2.0] Ha, each sorted ascending;
* antisymmetrised integrals <pq||rs> with standard deviation 0.05 Ha, exactly antisymmetric
  and Hermitian (see ``synth.c``);
* T1 iid N(0, 0.01^2); T2 MP2-like  t_ij^ab = <ij||ab> / (e_i + e_j - e_a - e_b);
* Lambda = T^dagger, i.e. l1 = t1 and l2 = t2 (all real).

Index convention: global spin-orbital index p < o is occupied, p = o + a is virtual a.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")

STREAM_EPS_OCC = 1
STREAM_EPS_VIR = 2
STREAM_T1 = 3
STREAM_ERI = 4

ERI_SCALE = 0.05
T1_SIGMA = 0.01
EPS_OCC = (-1.5, -0.3)
EPS_VIR = (0.1, 2.0)


def build(force: bool = False) -> str:
    """Compile ``libsynth.so`` with gcc (OpenMP). Returns the path."""
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        u64, i64, dbl, ptr = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.synth_uniform.argtypes = [u64, u64, i64, dbl, dbl, ptr]
        lib.synth_normal.argtypes = [u64, u64, i64, dbl, ptr]
        lib.synth_eri_block.argtypes = [u64, u64, dbl] + [i64] * 8 + [ptr]
        for f in (lib.synth_uniform, lib.synth_normal, lib.synth_eri_block):
            f.restype = None
        _lib = lib
    return _lib


def uniform(seed: int, stream: int, n: int, lo: float, hi: float) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_uniform(seed, stream, n, lo, hi, out.ctypes.data)
    return out


def normal(seed: int, stream: int, n: int, sigma: float) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_normal(seed, stream, n, sigma, out.ctypes.data)
    return out


def eri_range(seed: int, ranges, scale: float = ERI_SCALE) -> np.ndarray:
    """<pq||rs> for global index ranges ((p0,np),(q0,nq),(r0,nr),(s0,ns)); shape (np,nq,nr,ns)."""
    (p0, np_), (q0, nq), (r0, nr), (s0, ns) = ranges
    out = np.empty((np_, nq, nr, ns), dtype=np.float64)
    if out.size:
        _load().synth_eri_block(seed, STREAM_ERI, scale, p0, np_, q0, nq, r0, nr, s0, ns,
                                out.ctypes.data)
    return out


def eri_block(seed: int, o: int, v: int, kind: str, scale: float = ERI_SCALE) -> np.ndarray:
    """Integral block by occupancy pattern, e.g. ``"ovvo"`` -> <i a || b j> of shape (o,v,v,o)."""
    rng = {"o": (0, o), "v": (o, v)}
    return eri_range(seed, [rng[c] for c in kind], scale)


@dataclass
class Problem:
    """Synthetic inputs of one operator. Integral blocks are generated on first use."""

    o: int
    v: int
    seed: int
    eps: np.ndarray
    t1: np.ndarray
    blocks: dict = field(default_factory=dict)
    _t2: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.o + self.v

    def block(self, kind: str) -> np.ndarray:
        if kind not in self.blocks:
            self.blocks[kind] = eri_block(self.seed, self.o, self.v, kind)
        return self.blocks[kind]

    @property
    def t2(self) -> np.ndarray:
        """MP2-like doubles: <ij||ab> / (e_i + e_j - e_a - e_b), shape (o,o,v,v)."""
        if self._t2 is None:
            eo, ev = self.eps[: self.o], self.eps[self.o:]
            den = (eo[:, None, None, None] + eo[None, :, None, None]
                   - ev[None, None, :, None] - ev[None, None, None, :])
            self._t2 = self.block("oovv") / den
        return self._t2

    @property
    def l1(self) -> np.ndarray:
        return self.t1

    @property
    def l2(self) -> np.ndarray:
        return self.t2

    def full_eri(self) -> np.ndarray:
        """The whole (n,n,n,n) tensor; only for tiny models."""
        n = self.n
        return eri_range(self.seed, [(0, n)] * 4)


def make_problem(o: int, v: int, seed: int, t1_sigma: float = T1_SIGMA,
                 eri_scale: float = ERI_SCALE) -> Problem:
    eps = np.concatenate([np.sort(uniform(seed, STREAM_EPS_OCC, o, *EPS_OCC)),
                          np.sort(uniform(seed, STREAM_EPS_VIR, v, *EPS_VIR))])
    t1 = normal(seed, STREAM_T1, o * v, t1_sigma).reshape(o, v)
    p = Problem(o=o, v=v, seed=seed, eps=eps, t1=t1)
    if eri_scale != ERI_SCALE:
        raise ValueError("non-default integral scale is not supported")
    return p


# Workloads by their shapes (spin orbitals) and grids: the small case, the benzene/cc-pVDZ
# shape (plain solves, its reduced model, its adjoint gradient) and the adenine/cc-pVDZ shape
# (one batched mixed-precision block).
WORKLOADS = {
    "o10v20": dict(o=10, v=20, seed=0, omega=(-1.0, -0.3, 64), eta=0.01, np=10, tol=1e-10),
    "o42v186": dict(o=42, v=186, seed=1, omega=(-0.8, -0.2, 200), eta=0.005, np=8, tol=1e-10),
    "o42v186_mor": dict(o=42, v=186, seed=1, omega=(-0.9, -0.1, 4000), eta=0.005, np=8, tol=1e-10,
            sample_window=(-0.8, -0.2), per_round=8, resid_tol=1e-6,
            check=(-0.9, -0.1, 200)),
    "o70v260_mixed": dict(o=70, v=260, seed=3, omega=(-0.5, -0.3, 32), eta=0.005, np=16, tol=1e-8),
    "o42v186_adjoint": dict(o=42, v=186, seed=1, omega=(-0.6, -0.3, 100), eta=0.005, np=8, tol=1e-10),
}


def valence_p(o: int, np_: int) -> np.ndarray:
    """The np_ highest-energy occupied spin orbitals (energies are sorted ascending)."""
    return np.arange(o - np_, o, dtype=np.int32)


def omega_grid(spec) -> np.ndarray:
    lo, hi, n = spec
    return np.linspace(lo, hi, n)
