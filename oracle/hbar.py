"""Closed-form similarity-transformed Hamiltonian blocks used by the IP sigma product.

The paper (Methodology, definition of H-bar under Eq. gfxn1) defines H-bar = e^{-T} H e^{T}
but prints no matrix elements. The blocks below are the standard CCSD H-bar elements in a
spin-orbital basis with a diagonal Fock matrix f = diag(eps); each expression is checked
against the brute-force Fock-space construction in ``oracle.fock`` on tiny random models.

All arrays are full (unpacked) and antisymmetric where the indices say so. Integral blocks
follow the generator convention, e.g. ``ovvo[m, b, e, j] = <m b || e j>``.

Test infrastructure only: the product path never imports this package.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

def es(*args):
    return np.einsum(*args, optimize=True)


@dataclass
class HBar:
    o: int
    v: int
    Fov: np.ndarray   # F_me   [m, e]
    Foo: np.ndarray   # F_mi   [m, i]
    Fvv: np.ndarray   # F_ae   [a, e]
    Woooo: np.ndarray  # W_mnij [m, n, i, j]
    Wooov: np.ndarray  # W_mnie [m, n, i, e]
    Wovvo: np.ndarray  # W_mbej [m, b, e, j]
    Wovoo: np.ndarray  # W_mbij [m, b, i, j]
    oovv: np.ndarray   # <mn||ef> (bare; three-body term)
    t2: np.ndarray     # t_ij^ab (three-body term)


def tau(t1, t2):
    """tau_ij^ab = t_ij^ab + t_i^a t_j^b - t_i^b t_j^a."""
    return t2 + es("ia,jb->ijab", t1, t1) - es("ib,ja->ijab", t1, t1)


def build_hbar(o, v, eps, t1, t2, oooo, ooov, oovv, ovvo, ovvv) -> HBar:
    """H-bar blocks from the amplitudes and the five integral blocks.

    Integral identities used (all exact for an antisymmetric Hermitian real tensor):
    <am||ef> = -<ma||ef>,  <mb||ij> = <ij||mb>,  <mn||ej> = -<mn||je>.
    """
    eo = eps[:o]
    ev = eps[o:]
    ta = tau(t1, t2)
    # One-body blocks
    Fov = es("nf,mnef->me", t1, oovv)
    Foo = (np.diag(eo)
           + es("ne,mnie->mi", t1, ooov)
           + 0.5 * es("inef,mnef->mi", ta, oovv))
    Fvv = (np.diag(ev)
           - es("mf,maef->ae", t1, ovvv)  # t_m^f <am||ef>
           - 0.5 * es("mnaf,mnef->ae", ta, oovv))
    # Two-body blocks
    Woooo = (oooo
             + es("je,mnie->mnij", t1, ooov)
             - es("ie,mnje->mnij", t1, ooov)
             + 0.5 * es("ijef,mnef->mnij", ta, oovv))
    Wooov = ooov + es("if,mnfe->mnie", t1, oovv)
    Wovvo = (ovvo
             + es("jf,mbef->mbej", t1, ovvv)
             + es("nb,mnje->mbej", t1, ooov)          # -t_n^b <mn||ej>
             - es("jnfb,mnef->mbej", t2, oovv)
             - es("jf,nb,mnef->mbej", t1, t1, oovv))
    ovoo = ooov.transpose(2, 3, 0, 1)                  # <mb||ij> = <ij||mb>
    # <mb||ej> - t_nj^bf <mn||ef>
    Z = ovvo - es("njbf,mnef->mbej", t2, oovv)
    Wovoo = (ovoo
             - es("me,ijbe->mbij", Fov, t2)
             - es("nb,mnij->mbij", t1, Woooo)
             + 0.5 * es("mbef,ijef->mbij", ovvv, ta)
             + es("mnie,jnbe->mbij", ooov, t2)
             - es("mnje,inbe->mbij", ooov, t2)
             + es("ie,mbej->mbij", t1, Z)
             - es("je,mbei->mbij", t1, Z))
    return HBar(o=o, v=v, Fov=Fov, Foo=Foo, Fvv=Fvv, Woooo=Woooo, Wooov=Wooov, Wovvo=Wovvo,
                Wovoo=Wovoo, oovv=oovv, t2=t2)


def first_order_amplitudes(o, v, eps, oovv):
    """T and Lambda replaced by their first-order perturbative terms (the variant of the
    Conclusions, after Nooijen and Snijders), with the Moller-Plesset partitioning
    H0 = sum_p eps_p a+_p a_p of a diagonal Fock matrix: t1 = 0 (the singles coupling f_ia
    vanishes), t2_ij^ab = <ij||ab> / (e_i + e_j - e_a - e_b), and Lambda = T^dagger at this
    order (l1 = 0, l2 = t2 for real integrals). Returns (t1, t2, l1, l2)."""
    eo, ev = eps[:o], eps[o:]
    den = (eo[:, None, None, None] + eo[None, :, None, None]
           - ev[None, None, :, None] - ev[None, None, None, :])
    t2 = oovv / den
    z = np.zeros((o, v))
    return z, t2, z.copy(), t2.copy()


def build_hbar_first_order(prob) -> HBar:
    t1, t2, _, _ = first_order_amplitudes(prob.o, prob.v, prob.eps, prob.block("oovv"))
    return build_hbar(prob.o, prob.v, prob.eps, t1, t2, prob.block("oooo"), prob.block("ooov"),
                      prob.block("oovv"), prob.block("ovvo"), prob.block("ovvv"))


def build_hbar_from_problem(prob) -> HBar:
    return build_hbar(prob.o, prob.v, prob.eps, prob.t1, prob.t2, prob.block("oooo"),
                      prob.block("ooov"), prob.block("oovv"), prob.block("ovvo"),
                      prob.block("ovvv"))
