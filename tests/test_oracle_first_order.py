"""Pins of the first-order amplitudes (the perturbative T and Lambda variant of the Conclusions)
against brute-force Moller-Plesset perturbation theory in Fock space."""
import numpy as np
import pytest

import synth
from oracle import fock
from oracle import hbar as ohbar
from oracle import sigma as osig


@pytest.mark.parametrize("o,v,seed", [(2, 2, 1), (3, 3, 2), (4, 3, 3)])
def test_first_order_wavefunction_is_t_first_order(o, v, seed):
    """Rayleigh-Schrodinger theory with H0 = sum_p eps_p a+_p a_p gives the first-order
    wavefunction |Psi1> = sum_{K != Phi} |K> <K|H|Phi> / (E0_Phi - E0_K) in intermediate
    normalisation. It must equal T^(1)|Phi>: no singles, and doubles t2 of the closed form.
    The second-order energy <Phi|H|Psi1> is then 1/4 sum <ij||ab> t_ij^ab."""
    p = synth.make_problem(o, v, seed)
    eri = p.full_eri()
    n = o + v
    h = np.diag(p.eps) - np.einsum("piqi->pq", eri[:, :o, :, :o])
    ops = fock.Ops(n)
    H = fock.hamiltonian(ops, o, h, eri)
    dets, idx = fock.sector(n, o)
    e0 = np.array([sum(p.eps[q] for q in range(n) if d >> q & 1) for d in dets])
    ref = idx[(1 << o) - 1]
    phi = np.zeros(len(dets))
    phi[ref] = 1.0
    col = H @ phi
    psi1 = np.zeros(len(dets))
    for k in range(len(dets)):
        if k != ref:
            psi1[k] = col[k] / (e0[ref] - e0[k])
    t1, t2, l1, l2 = ohbar.first_order_amplitudes(o, v, p.eps, p.block("oovv"))
    T = fock.cluster(ops, o, o, t1, t2)
    assert np.abs(T @ phi - psi1).max() <= 1e-14 * np.abs(psi1).max()
    e2 = phi @ H @ psi1
    assert 0.25 * np.einsum("ijab,ijab->", p.block("oovv"), t2) == pytest.approx(e2, rel=1e-12)
    assert not t1.any() and not l1.any() and np.array_equal(l2, t2)


def test_first_order_operator_matches_brute_force():
    """The H-bar built from the first-order amplitudes is the brute-force similarity transform
    with those amplitudes (sigma, diagonal, b and c with Lambda = T^dagger)."""
    o, v = 3, 4
    p = synth.make_problem(o, v, 4)
    t1, t2, l1, l2 = ohbar.first_order_amplitudes(o, v, p.eps, p.block("oovv"))
    bf = fock.BruteForce(o, v, p.eps, t1, t2, p.full_eri(), l1=l1, l2=l2)
    M = bf.ip_matrix()
    hb = ohbar.build_hbar_first_order(p)
    D = osig.dim(o, v)
    dense = osig.sigma(hb, np.eye(D)).T
    assert np.abs(dense - M).max() <= 1e-12 * np.abs(M).max()
    assert np.abs(osig.diagonal(hb) - np.diag(M)).max() <= 1e-12 * np.abs(M).max()
    for q in range(o):
        assert np.abs(bf.c(q) - osig.c_vector(o, v, t1, t2, l1, l2, q)).max() < 1e-13


def test_first_order_amplitudes_are_the_recipes_doubles():
    """The synthetic doubles are already first order; the variant differs by T1 = Lambda1 = 0."""
    p = synth.make_problem(5, 6, 3)
    t1, t2, l1, l2 = ohbar.first_order_amplitudes(5, 6, p.eps, p.block("oovv"))
    assert np.array_equal(t2, p.t2)
    assert p.t1.any()
