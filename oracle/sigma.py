"""IP-EOM-CCSD sigma product, its transpose, the b and c vectors, G and A (closed forms).

The paper's auxiliary operator X_p (Eq. xp) has a one-hole part x^i and a two-hole-one-
particle part x^{ij}_a (i<j). The sigma product is the connected part of H-bar_N acting on it,
projected back onto that space (Eq. xplin and the definition of H-bar_N under Eq. gfxn1).
With r_ij^a antisymmetric in ij and P(ij) f_ij = f_ij - f_ji:

  sigma_i    = - F_ki r_k + F_ld r_il^d - 1/2 W_klid r_kl^d
  sigma_ij^a = - W_kaij r_k + F_ae r_ij^e - P(ij) F_ki r_kj^a + 1/2 W_klij r_kl^a
               + P(ij) W_maei r_mj^e - 1/2 <kl||cd> r_kl^c t_ij^ad

(repeated indices summed). Every term is checked against the brute-force Fock-space matrix.

Packed layout of a vector of length D = o + o(o-1)/2 * v: entries 0..o-1 hold x^i; entry
o + pi(i,j)*v + a holds x^{ij}_a for i<j with pi the lexicographic pair index.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

def es(*args):
    return np.einsum(*args, optimize=True)


def dim(o: int, v: int) -> int:
    return o + o * (o - 1) // 2 * v


def pair_index(o: int):
    """(iu, ju) arrays of the i<j pairs in lexicographic order."""
    iu, ju = np.triu_indices(o, k=1)
    return iu, ju


def unpack(x: np.ndarray, o: int, v: int):
    """Packed vector(s) [..., D] -> (r1 [..., o], r2 [..., o, o, v] antisymmetric)."""
    lead = x.shape[:-1]
    r1 = x[..., :o]
    iu, ju = pair_index(o)
    p2 = x[..., o:].reshape(lead + (len(iu), v))
    r2 = np.zeros(lead + (o, o, v), dtype=x.dtype)
    r2[..., iu, ju, :] = p2
    r2[..., ju, iu, :] = -p2
    return r1, r2


def pack(r1: np.ndarray, r2: np.ndarray) -> np.ndarray:
    o = r1.shape[-1]
    iu, ju = pair_index(o)
    p2 = r2[..., iu, ju, :]
    lead = r1.shape[:-1]
    return np.concatenate([r1, p2.reshape(lead + (-1,))], axis=-1)


def sigma_parts(hb, x: np.ndarray) -> dict:
    """Each of the nine sigma terms as a packed vector (for term-by-term checks)."""
    o, v = hb.o, hb.v
    r1, r2 = unpack(x, o, v)
    z1 = np.zeros_like(r1)
    z2 = np.zeros(r2.shape, dtype=r2.dtype)
    parts = {}
    parts["T1"] = pack(-es("ki,...k->...i", hb.Foo, r1), z2)
    parts["T2"] = pack(es("ld,...ild->...i", hb.Fov, r2), z2)
    parts["T3"] = pack(-0.5 * es("klid,...kld->...i", hb.Wooov, r2), z2)
    parts["T4"] = pack(z1, -es("kaij,...k->...ija", hb.Wovoo, r1))
    parts["T5"] = pack(z1, es("ae,...ije->...ija", hb.Fvv, r2))
    t6 = es("ki,...kja->...ija", hb.Foo, r2)
    parts["T6"] = pack(z1, -(t6 - np.swapaxes(t6, -3, -2)))
    parts["T7"] = pack(z1, 0.5 * es("klij,...kla->...ija", hb.Woooo, r2))
    t8 = es("maei,...mje->...ija", hb.Wovvo, r2)
    parts["T8"] = pack(z1, t8 - np.swapaxes(t8, -3, -2))
    tau_d = es("klcd,...klc->...d", hb.oovv, r2)
    parts["T9"] = pack(z1, -0.5 * es("ijad,...d->...ija", hb.t2, tau_d))
    return parts


def sigma(hb, x: np.ndarray) -> np.ndarray:
    """sigma = H-bar_N x for packed vector(s) x [..., D] (real or complex)."""
    return sum(sigma_parts(hb, x).values())


def sigma_t(hb, y: np.ndarray) -> np.ndarray:
    """Transpose product H-bar_N^T y, written term by term.

    Each term's adjoint is taken with respect to the packed dot product. With s2 the
    antisymmetric unpacked 2h1p part of y, that product is sum_i y_i s_i + 1/2 sum_ija, so
    the packed gradient of a bilinear form with respect to x_kl^c (k<l) is G_klc - G_lkc,
    where G is its derivative with respect to an unconstrained r_kl^c. ``g2`` below holds
    that antisymmetrised gradient for all (k, l); the packed result keeps k<l.
    """
    o, v = hb.o, hb.v
    s1, s2 = unpack(y, o, v)
    out1 = -es("ki,...i->...k", hb.Foo, s1)                       # T1
    out1 = out1 - 0.5 * es("kaij,...ija->...k", hb.Wovoo, s2)      # T4
    g2 = np.zeros(s2.shape, dtype=np.result_type(s2, hb.Fov))
    a2 = es("ld,...i->...ild", hb.Fov, s1)                         # T2
    g2 += a2 - np.swapaxes(a2, -3, -2)
    g2 -= es("klid,...i->...kld", hb.Wooov, s1)                    # T3
    g2 += es("ae,...ija->...ije", hb.Fvv, s2)                      # T5
    a6 = -es("ki,...ija->...kja", hb.Foo, s2)                      # T6
    g2 += a6 - np.swapaxes(a6, -3, -2)
    g2 += 0.5 * es("klij,...ija->...kla", hb.Woooo, s2)            # T7
    a8 = es("maei,...ija->...mje", hb.Wovvo, s2)                   # T8
    g2 += a8 - np.swapaxes(a8, -3, -2)
    u_d = es("ijad,...ija->...d", hb.t2, s2)                       # T9
    g2 -= 0.5 * es("klcd,...d->...klc", hb.oovv, u_d)
    return pack(out1, g2)


def diagonal(hb) -> np.ndarray:
    """Diagonal of H-bar_N in the packed basis (used for the Jacobi preconditioner)."""
    o, v = hb.o, hb.v
    D = dim(o, v)
    d = np.empty(D)
    d[:o] = -np.diag(hb.Foo)
    iu, ju = pair_index(o)
    Foo_d = np.diag(hb.Foo)
    Fvv_d = np.diag(hb.Fvv)
    # diagonal of each 2h1p term at (ij,a) <- (ij,a)
    dd = (Fvv_d[None, :]
          - Foo_d[iu][:, None] - Foo_d[ju][:, None]
          + hb.Woooo[iu, ju, iu, ju][:, None]
          + hb.Wovvo[iu[:, None], np.arange(v)[None, :], np.arange(v)[None, :], iu[:, None]]
          + hb.Wovvo[ju[:, None], np.arange(v)[None, :], np.arange(v)[None, :], ju[:, None]]
          - es("ijad,ijad->ija", hb.t2, hb.oovv)[iu, ju, :])
    d[o:] = dd.reshape(-1)
    return d


def b_vector(o: int, v: int, p: int) -> np.ndarray:
    """Right-hand side of Eq. xplin for an occupied p: a_p commutes with T, so b = e_p."""
    if not 0 <= p < o:
        raise ValueError("only occupied p are supported")
    b = np.zeros(dim(o, v))
    b[p] = 1.0
    return b


def c_vector(o: int, v: int, t1, t2, l1, l2, q: int) -> np.ndarray:
    """Row c_q of Eq. gfcclineqn: <Phi|(1 + Lambda_1 + Lambda_2) e^{-T} a+_q e^{T} (Eq. gfxn2).

    For occupied q = j:
      c_k      = delta_jk - l_k^a t_j^a - 1/2 l_kl^ab t_jl^ab
      c_kl^c   = delta_jk l_l^c - delta_jl l_k^c - t_j^a l_kl^ac          (k<l)
    """
    if not 0 <= q < o:
        raise ValueError("only occupied q are supported")
    c1 = -es("ka,a->k", l1, t1[q]) - 0.5 * es("klab,lab->k", l2, t2[q])
    c1[q] += 1.0
    c2 = np.zeros((o, o, v))
    c2[q, :, :] += l1
    c2[:, q, :] -= l1
    c2 -= es("a,klac->klc", t1[q], l2)
    return pack(c1, c2)
