"""torch.autograd wrapper of the windowed spectral weight and its hand-written adjoint.

J(eps) = sum_k w_k A(omega_k), A(omega) = (1/pi) sum_p Im G_pp(omega). The forward pass builds
the operator for the given orbital energies and solves the shifted systems (libgfcc.so); the
backward pass solves the transposed systems (omega - i eta + H-bar_N^T) y_p = c_p and reduces
dJ/deps_r = (1/pi) sum_k w_k sum_p Im(-y_p^T D_r x_p) on the device (gfcc_grad_eps), with
D_r = dH-bar_N/deps_r at fixed amplitudes.
"""
from __future__ import annotations

import torch

from . import gfcc


class SpectralWeight(torch.autograd.Function):
    """SpectralWeight.apply(eps, ctx, inputs, omega, weights, p, eta, tol) -> J (0-d tensor).

    eps: float64 tensor [o+v] on the context's device (the differentiated input).
    inputs: dict of the other device tensors of build_hbar_operands (t1, t2, l1, l2, oooo,
    ooov, oovv, ovvo, ovvv), held fixed.
    """

    @staticmethod
    def forward(fctx, eps, gctx: gfcc.Context, inputs: dict, omega, weights, p, eta, tol):
        o, v = inputs["t1"].shape
        e = eps.detach().contiguous()
        gctx.build_hbar_operands(o, v, e, inputs["t1"], inputs["t2"], inputs["l1"], inputs["l2"],
                                 inputs["oooo"], inputs["ooov"], inputs["oovv"], inputs["ovvo"],
                                 inputs["ovvv"])
        res = gctx.gfcc_solve(omega, p, eta, tol=tol, want_x=True)
        J = gfcc.spectral_weight(res.G, weights)
        fctx.gctx, fctx.X = gctx, res.X
        fctx.args = (omega, weights, p, eta, tol)
        fctx.eps_dev = eps.device
        return torch.tensor(J, dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(fctx, grad_out):
        omega, weights, p, eta, tol = fctx.args
        adj = fctx.gctx.gfcc_solve(omega, p, eta, tol=tol, transpose=True, want_x=True)
        g = fctx.gctx.gfcc_grad_eps(weights, fctx.X, adj.X)
        grad = torch.from_numpy(g).to(fctx.eps_dev) * grad_out
        return grad, None, None, None, None, None, None, None
