"""FP64 iterative refinement around a reduced-precision GMRES (GMRES-IR). Test infrastructure.

Outer loop in FP64: r = b - M x; stop when ||r||/||b|| <= tol; otherwise solve M d = r
approximately with an inner GMRES whose sigma product runs in FP32 (and, optionally, with the
three-body term's operands rounded to bfloat16), then x += d. The inner Arnoldi, Givens
rotations and least-squares solves stay in FP64. (Carson & Higham's GMRES-IR scheme.)

The reduced-precision sigma is emulated with float32 copies of the operator blocks and
float32 arithmetic; bfloat16 rounding is round-to-nearest-even on the float32 bit pattern.
The three-body term's bfloat16 operands are two-term values x = hi + lo (hi = bf16(x),
lo = bf16(x - hi)), and each of its two products is hi.hi + hi.lo + lo.hi accumulated in
float32: the products run on bfloat16 inputs while the term keeps about 16 significant bits.
With pairs=True the terms that contract the 2h1p block with Fvv, Foo and Wovvo are formed the
same way (each block and the vector split into two-term pairs) instead.
"""
from __future__ import annotations

import copy

import numpy as np

from . import sigma as sg
from . import solve as so


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def bf16_split(x: np.ndarray):
    """x (float32 or float64) as hi + lo: hi = bf16(x), lo = bf16(x - hi), both float32."""
    a = np.asarray(x)
    hi = bf16_round(a.astype(np.float32))
    lo = bf16_round((a - hi.astype(a.dtype)).astype(np.float32))
    return hi, lo


def f32_hbar(hb):
    h = copy.copy(hb)
    for name in ("Fov", "Foo", "Fvv", "Woooo", "Wooov", "Wovvo", "Wovoo", "oovv", "t2"):
        setattr(h, name, getattr(hb, name).astype(np.float32))
    return h


def _pair_product(spec, a, b):
    """a.b on two-term bf16 operands: ah.bh + ah.bl + al.bh in float32."""
    ah, al = bf16_split(a)
    bh, bl = bf16_split(b)
    return (np.einsum(spec, ah, bh) + np.einsum(spec, ah, bl)
            + np.einsum(spec, al, bh)).astype(np.float32)


def sigma_reduced(h32, x: np.ndarray, bf16_3body: bool, pairs: bool = False) -> np.ndarray:
    """sigma in float32 (complex64) arithmetic; three-body operands optionally in bf16.

    pairs: the terms that contract the 2h1p block with Fvv, Foo and Wovvo (T5, T6, T8 of the
    IP sigma) on two-term bf16 operands."""
    xr = x.real.astype(np.float32)
    xi = x.imag.astype(np.float32)
    out = []
    for part in (xr, xi):
        parts = sg.sigma_parts(h32, part)
        if pairs:
            o = h32.o
            _, r2 = sg.unpack(part, o, h32.v)
            z1 = np.zeros(part.shape[:-1] + (o,), np.float32)
            parts["T5"] = sg.pack(z1, _pair_product("ae,...ije->...ija", h32.Fvv, r2))
            t6 = _pair_product("ki,...kja->...ija", h32.Foo, r2)
            parts["T6"] = sg.pack(z1, -(t6 - np.swapaxes(t6, -3, -2)))
            t8 = _pair_product("maei,...mje->...ija", h32.Wovvo, r2)
            parts["T8"] = sg.pack(z1, t8 - np.swapaxes(t8, -3, -2))
        if bf16_3body:
            o, v = h32.o, h32.v
            xh, xl = bf16_split(part)
            _, rh = sg.unpack(xh, o, v)
            _, rl = sg.unpack(xl, o, v)
            vh, vl = bf16_split(h32.oovv)
            tau = (np.einsum("klcd,...klc->...d", vh, rh) + np.einsum("klcd,...klc->...d", vh, rl)
                   + np.einsum("klcd,...klc->...d", vl, rh)).astype(np.float32)
            th, tl = bf16_split(h32.t2)
            uh, ul = bf16_split(tau)
            t9 = -0.5 * (np.einsum("ijad,...d->...ija", th, uh) + np.einsum("ijad,...d->...ija", th, ul)
                         + np.einsum("ijad,...d->...ija", tl, uh))
            parts["T9"] = sg.pack(np.zeros(part.shape[:-1] + (o,), np.float32), t9.astype(np.float32))
        out.append(sum(parts.values()).astype(np.float32))
    return out[0].astype(np.float64) + 1j * out[1].astype(np.float64)


class ReducedOperator(so.Operator):
    def __init__(self, hb, bf16_3body: bool, pairs: bool = False):
        super().__init__(hb)
        self.h32 = f32_hbar(hb)
        self.bf16 = bf16_3body
        self.pairs = pairs

    def hbar(self, x):
        self.nmatvec += 1
        return sigma_reduced(self.h32, x, self.bf16, self.pairs)


def gmres_ir(hb, b, omega, eta, tol=1e-8, inner_tol=1e-4, inner_maxit=100, restart=50,
             max_outer=30, bf16_3body=True, pairs=False):
    """Returns (x, outer steps, total inner iterations, final FP64 relative residual)."""
    op64 = so.Operator(hb)
    lo = ReducedOperator(hb, bf16_3body, pairs)
    shift = omega - 1j * eta
    x = np.zeros(op64.D, dtype=complex)
    bn = np.linalg.norm(b)
    inner_total = 0
    for outer in range(max_outer + 1):
        r = b - (op64.hbar(x) + shift * x)
        rel = np.linalg.norm(r) / bn
        if rel <= tol or outer == max_outer:
            return x, outer, inner_total, rel
        d, its, _ = so.gmres(lo, r, omega, eta, tol=inner_tol, restart=restart, maxit=inner_maxit)
        inner_total += its
        x = x + d
    return x, max_outer, inner_total, rel
