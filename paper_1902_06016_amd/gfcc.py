"""Python binding of libgfcc.so (ctypes). Argument marshalling only.

Every computation runs in the library's HIP kernels; torch is used for device memory (tensor
storage passed by pointer) and for the stream handle. Names follow the C ABI in
``include/gfcc.h``. Importing this module loads the library and raises if it is missing: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfcc.so")

GFCC_OK, GFCC_EINVAL, GFCC_ENOMEM, GFCC_EHIP, GFCC_ENOCONV, GFCC_EBREAKDOWN, GFCC_ESTATE = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ENOCONV", 5: "EBREAKDOWN",
                6: "ESTATE"}
FP64, FP32, FP32_BF16_3BODY, BF16_PAIRS = 0, 1, 2, 3
KEEP_FP64, KEEP_FP32, KEEP_TRANSPOSE = 1, 2, 4
EXPORT_BLOCKS = {"Foo": 0, "Fov": 1, "Fvv": 2, "Woooo": 3, "Wooov": 4, "Wovvo": 5, "Wovoo": 6,
                 "diag": 7}


class GfccError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1902_06016_amd.build`")
    # torch first: it loads the HIP runtime its wheel carries, and the library then binds to
    # that one (same soname). Loaded first, the library would bring in the system runtime and
    # torch a second copy of its own, and each would hold its own device state (contexts
    # fail, torch's streams are foreign to the library).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "gfcc_dim": (i64, [i32, i32]),
        "gfcc_create": (i32, [P(vp), i32, vp]),
        "gfcc_destroy": (i32, [vp]),
        "gfcc_last_error": (ctypes.c_char_p, [vp]),
        "build_hbar_operands": (i32, [vp, i32, i32] + [vp] * 10 + [i32]),
        "build_hbar_first_order": (i32, [vp, i32, i32] + [vp] * 6 + [i32]),
        "sigma_apply": (i32, [vp, i32, vp, vp, i32, i32]),
        "gfcc_solve": (i32, [vp, i32, vp, i32, vp, dbl, dbl, i32, i32, i32, i32, i32, vp, vp, vp,
                             vp]),
        "gfcc_solve_x0": (i32, [vp, i32, vp, i32, vp, dbl, dbl, i32, i32, i32, i32, i32, vp, vp,
                                vp, vp, vp]),
        "gfcc_solve_diis": (i32, [vp, i32, vp, i32, vp, dbl, dbl, i32, i32, i32, i32, vp, vp,
                                  vp, vp, vp, vp]),
        "gfcc_autotune": (i32, [vp, i32]),
        "gfcc_autotune_entry": (i32, [vp, i32, vp, vp]),
        "gfcc_autotune_pin": (i32, [vp, i32, i32, i32, i32]),
        "gfcc_graphs": (i32, [vp, i32]),
        "gfcc_compact": (i32, [vp, i32]),
        "gfcc_grad_eps": (i32, [vp, i32, vp, i32, vp, vp, vp]),
        "mor_build": (i32, [vp, i32, vp, i32, vp, dbl, dbl, dbl, P(vp)]),
        "mor_build_diag": (i32, [vp, i32, vp, i32, vp, dbl, dbl, dbl, vp]),
        "mor_refine": (i32, [vp, i32, vp, dbl, dbl, i32, dbl, i32, i32, vp, vp]),
        "mor_eval": (i32, [vp, i32, vp, vp, vp]),
        "mor_eval_noalloc": (i32, [vp, i32, vp, vp, vp]),
        "mor_lift": (i32, [vp, i32, vp, vp]),
        "mor_info": (i32, [vp, vp, vp, vp, i32]),
        "mor_destroy": (i32, [vp]),
        "spectral_function": (i32, [i32, i32, vp, i32, vp]),
        "spectral_weight": (i32, [i32, i32, vp, i32, vp, vp]),
        "gfcc_export": (i32, [vp, i32, vp]),
        "gfcc_timer": (i32, [vp, i32, i32, i32, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()
SYMBOLS = ("gfcc_dim", "gfcc_create", "gfcc_destroy", "gfcc_last_error", "build_hbar_operands",
           "build_hbar_first_order", "sigma_apply", "gfcc_autotune", "gfcc_autotune_entry",
           "gfcc_autotune_pin", "gfcc_graphs", "gfcc_compact",
           "gfcc_solve", "gfcc_solve_x0", "gfcc_solve_diis", "gfcc_grad_eps", "mor_build",
           "mor_build_diag", "mor_refine", "mor_eval", "mor_eval_noalloc", "mor_lift",
           "mor_info", "mor_destroy", "spectral_function", "spectral_weight", "gfcc_export",
           "gfcc_timer")


def dim(o: int, v: int) -> int:
    return int(lib.gfcc_dim(o, v))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _f64arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _i32arr(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class SolveResult:
    G: object            # torch complex128 [nw][np][np] (device)
    X: object | None     # torch complex128 [nw][np][D] (device) or None
    iters: np.ndarray    # [nw, np]
    resid: np.ndarray    # [nw, np]
    status: int
    hist: np.ndarray | None = None   # DIIS: [nw, np, maxit + 1] residual histories, -1 padded


class Context:
    """A library context bound to one HIP device and torch's current stream on it."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(lib.gfcc_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)),
                    ctx=None)
        self.h = h
        self.o = self.v = self.D = None
        self._models = weakref.WeakSet()

    def _check(self, st, ctx="self", allow=()):
        if st != GFCC_OK and st not in allow:
            msg = lib.gfcc_last_error(self.h if ctx == "self" else None) or b""
            raise GfccError(st, msg.decode())
        return st

    def close(self):
        """Free the context; models built on it are freed first (they point into it)."""
        if getattr(self, "h", None) is not None and self.h.value:
            for m in list(getattr(self, "_models", ())):
                m.close()
            lib.gfcc_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- operator
    def build_hbar_operands(self, o, v, eps, t1, t2, l1, l2, oooo, ooov, oovv, ovvo, ovvv,
                            keep: int = KEEP_FP64):
        """All arrays: torch float64 tensors on this context's device (contiguous)."""
        arrs = [eps, t1, t2, l1, l2, oooo, ooov, oovv, ovvo, ovvv]
        for a in arrs:
            if a.dtype != self.torch.float64 or not a.is_contiguous() or a.device != self.device:
                raise ValueError("build_hbar_operands expects contiguous float64 device tensors")
        self._check(lib.build_hbar_operands(self.h, o, v, *[_ptr(a) for a in arrs], keep))
        self.o, self.v, self.D = o, v, dim(o, v)

    def build_hbar_first_order(self, o, v, eps, oooo, ooov, oovv, ovvo, ovvv,
                               keep: int = KEEP_FP64):
        """The operator from first-order amplitudes formed on the device; arrays as in
        build_hbar_operands."""
        arrs = [eps, oooo, ooov, oovv, ovvo, ovvv]
        for a in arrs:
            if a.dtype != self.torch.float64 or not a.is_contiguous() or a.device != self.device:
                raise ValueError("build_hbar_first_order expects contiguous float64 device tensors")
        self._check(lib.build_hbar_first_order(self.h, o, v, *[_ptr(a) for a in arrs], keep))
        self.o, self.v, self.D = o, v, dim(o, v)

    def build_first_order_from_problem(self, prob, keep: int = KEEP_FP64):
        """Upload a synthetic problem's energies and integrals (no amplitudes) and build the
        operator from first-order amplitudes."""
        T = self.torch
        arrs = [prob.eps] + [prob.block(k) for k in ("oooo", "ooov", "oovv", "ovvo", "ovvv")]
        dev = [T.from_numpy(np.ascontiguousarray(a)).to(self.device) for a in arrs]
        self.build_hbar_first_order(prob.o, prob.v, *dev, keep=keep)
        del dev
        T.cuda.synchronize(self.device)

    def build_from_problem(self, prob, keep: int = KEEP_FP64):
        """Upload a synthetic problem (``synth.Problem``) and build the operator from it."""
        T = self.torch

        def up(a):
            return T.from_numpy(np.ascontiguousarray(a)).to(self.device)

        arrs = [prob.eps, prob.t1, prob.t2, prob.l1, prob.l2] + [
            prob.block(k) for k in ("oooo", "ooov", "oovv", "ovvo", "ovvv")]
        dev = [up(a) for a in arrs]
        self.build_hbar_operands(prob.o, prob.v, *dev, keep=keep)
        del dev
        T.cuda.synchronize(self.device)

    def export(self, name: str):
        o, v, D = self.o, self.v, self.D
        shapes = {"Foo": (o, o), "Fov": (o, v), "Fvv": (v, v), "Woooo": (o, o, o, o),
                  "Wooov": (o, o, o, v), "Wovvo": (o, v, v, o), "Wovoo": (o, v, o, o), "diag": (D,)}
        out = self.torch.empty(shapes[name], dtype=self.torch.float64, device=self.device)
        self._check(lib.gfcc_export(self.h, EXPORT_BLOCKS[name], _ptr(out)))
        return out

    # ------------------------------------------------------------------ sigma
    def sigma_apply(self, x, transpose: bool = False, precision: int = FP64):
        """x: complex128 [nrhs][D] device tensor -> Hbar_N x (or Hbar_N^T x)."""
        x = x.contiguous()
        if x.dtype != self.torch.complex128 or x.dim() != 2 or x.shape[1] != self.D:
            raise ValueError("sigma_apply expects complex128 [nrhs][D]")
        y = self.torch.empty_like(x)
        self._check(lib.sigma_apply(self.h, x.shape[0], _ptr(x), _ptr(y), int(transpose), precision))
        return y

    # ------------------------------------------------------------------ solve
    def gfcc_solve(self, omega, p, eta, tol=1e-10, maxit=500, restart=30, block=0,
                   precision=FP64, transpose=False, want_x=False, allow_noconv=False, x0=None):
        """x0: optional initial guesses, complex128 [nw][np][D] device tensor (gfcc_solve_x0)."""
        om, om_p = _f64arr(omega)
        pp, p_p = _i32arr(p)
        nw, np_ = len(om), len(pp)
        T = self.torch
        G = T.empty((nw, np_, np_), dtype=T.complex128, device=self.device)
        X = T.empty((nw, np_, self.D), dtype=T.complex128, device=self.device) if want_x else None
        its = np.zeros(nw * np_, dtype=np.int32)
        res = np.zeros(nw * np_, dtype=np.float64)
        xp = _ptr(X) if X is not None else None
        ip, rp = its.ctypes.data_as(ctypes.c_void_p), res.ctypes.data_as(ctypes.c_void_p)
        if x0 is None:
            st = lib.gfcc_solve(self.h, nw, om_p, np_, p_p, eta, tol, maxit, restart, block,
                                precision, int(transpose), xp, _ptr(G), ip, rp)
        else:
            x0 = x0.contiguous()
            if x0.dtype != T.complex128 or tuple(x0.shape) != (nw, np_, self.D):
                raise ValueError("x0 must be complex128 [nw][np][D]")
            st = lib.gfcc_solve_x0(self.h, nw, om_p, np_, p_p, eta, tol, maxit, restart, block,
                                   precision, int(transpose), _ptr(x0), xp, _ptr(G), ip, rp)
        self._check(st, allow=(GFCC_ENOCONV,) if allow_noconv else ())
        return SolveResult(G=G, X=X, iters=its.reshape(nw, np_), resid=res.reshape(nw, np_), status=st)

    def gfcc_solve_diis(self, omega, p, eta, tol=1e-10, maxit=500, ndiis=10, block=0,
                        transpose=False, want_x=False, allow_noconv=False, x0=None,
                        want_hist=False):
        """Complex DIIS solves (gfcc_solve_diis); x0 as in gfcc_solve."""
        om, om_p = _f64arr(omega)
        pp, p_p = _i32arr(p)
        nw, np_ = len(om), len(pp)
        T = self.torch
        G = T.empty((nw, np_, np_), dtype=T.complex128, device=self.device)
        X = T.empty((nw, np_, self.D), dtype=T.complex128, device=self.device) if want_x else None
        its = np.zeros(nw * np_, dtype=np.int32)
        res = np.zeros(nw * np_, dtype=np.float64)
        hist = np.zeros((nw, np_, maxit + 1), dtype=np.float64) if want_hist else None
        if x0 is not None:
            x0 = x0.contiguous()
            if x0.dtype != T.complex128 or tuple(x0.shape) != (nw, np_, self.D):
                raise ValueError("x0 must be complex128 [nw][np][D]")
        st = lib.gfcc_solve_diis(self.h, nw, om_p, np_, p_p, eta, tol, maxit, ndiis, block,
                                 int(transpose), _ptr(x0) if x0 is not None else None,
                                 _ptr(X) if X is not None else None, _ptr(G),
                                 its.ctypes.data_as(ctypes.c_void_p),
                                 res.ctypes.data_as(ctypes.c_void_p),
                                 hist.ctypes.data_as(ctypes.c_void_p) if hist is not None else None)
        self._check(st, allow=(GFCC_ENOCONV,) if allow_noconv else ())
        return SolveResult(G=G, X=X, iters=its.reshape(nw, np_), resid=res.reshape(nw, np_),
                           status=st, hist=hist)

    def gfcc_grad_eps(self, weight, X, Y):
        w, w_p = _f64arr(weight)
        out = np.zeros(self.o + self.v)
        self._check(lib.gfcc_grad_eps(self.h, len(w), w_p, X.shape[1], _ptr(X.contiguous()),
                                      _ptr(Y.contiguous()), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    # ------------------------------------------------------------- autotuner
    def autotune(self, enable=True):
        """enable: False/0 off, True/1 timed, 2 the most split variant of every class untimed."""
        self._check(lib.gfcc_autotune(self.h, int(enable)))

    def graphs(self, enable: bool = True):
        """Capture the Arnoldi steps of small blocks as HIP graphs (gfcc_graphs)."""
        self._check(lib.gfcc_graphs(self.h, int(enable)))

    def compact(self, enable: bool = True):
        """Continue the right-hand sides a GMRES restart leaves active in a compacted block
        (gfcc_compact)."""
        self._check(lib.gfcc_compact(self.h, int(enable)))

    def autotune_pin(self, kind: int, tile_m: int, tile_n: int, splits: int = 1):
        """Fix the choice of one of the sigma's fused product kinds (20/21); tile (0, 0) = the
        unfused route."""
        self._check(lib.gfcc_autotune_pin(self.h, kind, tile_m, tile_n, splits))

    def autotune_entries(self):
        """The tuner's choices: dicts with the product kind (0/1 plain product with transA,
        20/21 the sigma's fused products), shape, split count (0 = generic kernel), tile
        (0 x 0: a plain product, or the unfused sigma route) and the measured times."""
        out = []
        desc = (ctypes.c_int64 * 8)()
        us = (ctypes.c_double * 2)()
        i = 0
        while lib.gfcc_autotune_entry(self.h, i, desc, us) == GFCC_OK:
            out.append({"elem_bytes": desc[0], "kind": desc[1], "transA": desc[1] == 1,
                        "M": desc[2], "N": desc[3], "K": desc[4], "splits": desc[5],
                        "tile": (desc[6], desc[7]), "us": us[0], "generic_us": us[1]})
            i += 1
        return out

    # ---------------------------------------------------------------- timers
    def timer(self, which: int, enable: bool = True, reset: bool = True):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib.gfcc_timer(self.h, which, int(enable), int(reset), ctypes.byref(ms),
                                   ctypes.byref(n)))
        return ms.value, n.value

    # -------------------------------------------------------------------- MOR
    def mor_build(self, omega_k, p, eta, solve_tol=1e-10, defl_tol=1e-10):
        om, om_p = _f64arr(omega_k)
        pp, p_p = _i32arr(p)
        h = ctypes.c_void_p()
        self._check(lib.mor_build(self.h, len(om), om_p, len(pp), p_p, eta, solve_tol, defl_tol,
                                  ctypes.byref(h)))
        model = MorModel(self, h, len(pp))
        self._models.add(model)
        return model

    def mor_build_diag(self, omega_k, p, eta, solve_tol=1e-10, defl_tol=1e-10):
        """One reduced model per orbital of p (each for its diagonal G_pp), sharing the full
        solves; returns the list of models in the order of p."""
        om, om_p = _f64arr(omega_k)
        pp, p_p = _i32arr(p)
        hs = (ctypes.c_void_p * len(pp))()
        self._check(lib.mor_build_diag(self.h, len(om), om_p, len(pp), p_p, eta, solve_tol,
                                       defl_tol, ctypes.cast(hs, ctypes.c_void_p)))
        models = []
        for h in hs:
            model = MorModel(self, ctypes.c_void_p(h), 1)
            self._models.add(model)
            models.append(model)
        return models


class MorModel:
    """A reduced-order model owned by the library (freed on close / garbage collection)."""

    def __init__(self, ctx: Context, h, np_: int):
        self.ctx, self.h, self.np = ctx, h, np_

    def refine(self, grid, wmin, wmax, per_round=8, resid_tol=1e-6, max_order=4096, max_rounds=20):
        g, g_p = _f64arr(grid)
        rounds = ctypes.c_int()
        mres = ctypes.c_double()
        st = lib.mor_refine(self.h, len(g), g_p, wmin, wmax, per_round, resid_tol, max_order,
                            max_rounds, ctypes.byref(rounds), ctypes.byref(mres))
        self.ctx._check(st)
        return rounds.value, mres.value

    def eval(self, omega, want_resid=True):
        om, om_p = _f64arr(omega)
        T = self.ctx.torch
        G = T.empty((len(om), self.np, self.np), dtype=T.complex128, device=self.ctx.device)
        res = np.zeros(len(om)) if want_resid else None
        st = lib.mor_eval(self.h, len(om), om_p, _ptr(G),
                          res.ctypes.data_as(ctypes.c_void_p) if want_resid else None)
        self.ctx._check(st)
        return G, res

    def lift(self, omega):
        """Full-space approximate solutions S xhat_p(omega): complex128 [nw][np][D] (device)."""
        om, om_p = _f64arr(omega)
        T = self.ctx.torch
        X = T.empty((len(om), self.np, self.ctx.D), dtype=T.complex128, device=self.ctx.device)
        self.ctx._check(lib.mor_lift(self.h, len(om), om_p, _ptr(X)))
        return X

    def info(self, cap=4096):
        m = ctypes.c_int()
        nk = ctypes.c_int()
        oks = np.zeros(cap)
        self.ctx._check(lib.mor_info(self.h, ctypes.byref(m), ctypes.byref(nk),
                                     oks.ctypes.data_as(ctypes.c_void_p), cap))
        return m.value, oks[: min(nk.value, cap)].copy()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib.mor_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spectral_function(G) -> np.ndarray:
    """A(omega) = (1/pi) sum_p Im G_pp for G complex128 [nw][np][np] (torch device tensor or
    numpy host array)."""
    if isinstance(G, np.ndarray):
        g = np.ascontiguousarray(G, dtype=np.complex128)
        out = np.zeros(g.shape[0])
        st = lib.spectral_function(g.shape[0], g.shape[1], g.ctypes.data_as(ctypes.c_void_p), 0,
                                   out.ctypes.data_as(ctypes.c_void_p))
    else:
        g = G.contiguous()
        out = np.zeros(g.shape[0])
        st = lib.spectral_function(g.shape[0], g.shape[1], _ptr(g), 1,
                                   out.ctypes.data_as(ctypes.c_void_p))
    if st != GFCC_OK:
        raise GfccError(st, "spectral_function failed")
    return out


def spectral_weight(G, weight) -> float:
    """J = sum_w weight_w A(omega_w) for G complex128 [nw][np][np] (torch device tensor or numpy
    host array) and host weights [nw]."""
    w, w_p = _f64arr(weight)
    J = ctypes.c_double()
    if isinstance(G, np.ndarray):
        g = np.ascontiguousarray(G, dtype=np.complex128)
        st = lib.spectral_weight(g.shape[0], g.shape[1], g.ctypes.data_as(ctypes.c_void_p), 0,
                                 w_p, ctypes.byref(J))
    else:
        g = G.contiguous()
        st = lib.spectral_weight(g.shape[0], g.shape[1], _ptr(g), 1, w_p, ctypes.byref(J))
    if st != GFCC_OK:
        raise GfccError(st, "spectral_weight failed")
    return J.value
