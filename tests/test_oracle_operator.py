"""Pins of the closed-form operator (H-bar blocks, sigma, sigma^T, b, c) against the brute-force
Fock-space construction and against special cases with known answers."""
import copy

import numpy as np
import pytest

import synth
from oracle import fock
from oracle import hbar as ohbar
from oracle import sigma as osig


def _model(o, v, seed, t1s=0.2, t2s=5.0, lam=False):
    p = synth.make_problem(o, v, seed)
    eri = p.full_eri()
    t1 = synth.normal(seed, 9, o * v, t1s).reshape(o, v)
    t2 = p.t2 * t2s
    if lam:
        l1 = synth.normal(seed, 10, o * v, t1s).reshape(o, v)
        l2 = -3.0 * p.t2
    else:
        l1, l2 = t1, t2
    return p, eri, t1, t2, l1, l2


def _closed(p, t1, t2, eps=None):
    b = p.block
    return ohbar.build_hbar(p.o, p.v, p.eps if eps is None else eps, t1, t2, b("oooo"),
                            b("ooov"), b("oovv"), b("ovvo"), b("ovvv"))


def _dense(hb, fn=osig.sigma):
    D = osig.dim(hb.o, hb.v)
    return fn(hb, np.eye(D)).T


CASES = [(2, 1, 1), (2, 3, 2), (3, 2, 3), (3, 4, 4), (4, 3, 5), (4, 4, 6)]


@pytest.mark.parametrize("o,v,seed", CASES)
def test_sigma_matches_brute_force(o, v, seed):
    p, eri, t1, t2, l1, l2 = _model(o, v, seed, lam=True)
    bf = fock.BruteForce(o, v, p.eps, t1, t2, eri, l1=l1, l2=l2)
    M = bf.ip_matrix()
    hb = _closed(p, t1, t2)
    scale = np.abs(M).max()
    assert np.abs(_dense(hb) - M).max() < 1e-12 * scale
    assert np.abs(_dense(hb, osig.sigma_t) - M.T).max() < 1e-12 * scale
    assert np.abs(osig.diagonal(hb) - np.diag(M)).max() < 1e-12 * scale
    for q in range(o):
        assert np.abs(bf.b(q) - osig.b_vector(o, v, q)).max() < 1e-14
        assert np.abs(bf.c(q) - osig.c_vector(o, v, t1, t2, l1, l2, q)).max() < 1e-13


def test_every_term_and_block_is_load_bearing():
    """A plausible mistake anywhere (a dropped term, a perturbed block) breaks the pin."""
    o, v, seed = 4, 3, 8
    p, eri, t1, t2, _, _ = _model(o, v, seed)
    M = fock.BruteForce(o, v, p.eps, t1, t2, eri).ip_matrix()
    hb = _closed(p, t1, t2)
    D = osig.dim(o, v)
    parts = osig.sigma_parts(hb, np.eye(D))
    for k in parts:
        wrong = sum(val for kk, val in parts.items() if kk != k).T
        assert np.abs(wrong - M).max() > 1e-3, k
    rng = np.random.default_rng(0)
    for name in ("Foo", "Fov", "Fvv", "Woooo", "Wooov", "Wovvo", "Wovoo", "oovv", "t2"):
        h2 = copy.copy(hb)
        setattr(h2, name, getattr(hb, name) + 1e-3 * rng.standard_normal(getattr(hb, name).shape))
        assert np.abs(_dense(h2) - M).max() > 1e-6, name


def test_noninteracting_limit():
    """T = 0 and no two-electron integrals: diagonal -eps_i and eps_a - eps_i - eps_j."""
    o, v = 3, 4
    p = synth.make_problem(o, v, 1)
    z = np.zeros
    hb = ohbar.build_hbar(o, v, p.eps, z((o, v)), z((o, o, v, v)), z((o,) * 4), z((o, o, o, v)),
                          z((o, o, v, v)), z((o, v, v, o)), z((o, v, v, v)))
    Hd = _dense(hb)
    iu, ju = osig.pair_index(o)
    eo, ev = p.eps[:o], p.eps[o:]
    expect = np.concatenate([-eo, (ev[None, :] - eo[iu][:, None] - eo[ju][:, None]).ravel()])
    assert np.abs(Hd - np.diag(expect)).max() < 1e-14


def test_t_zero_gives_symmetric_ip_matrix():
    """With T = 0 the IP block is the Hermitian 2h1p-TDA/CI matrix of H."""
    o, v = 4, 3
    p = synth.make_problem(o, v, 3)
    eri = p.full_eri()
    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    M = fock.BruteForce(o, v, p.eps, z1, z2, eri).ip_matrix()
    assert np.abs(M - M.T).max() < 1e-14
    hb = _closed(p, z1, z2)
    assert np.abs(_dense(hb) - M).max() < 1e-13


def test_commutator_removes_energy_and_residual():
    """<Phi_mu|H-bar|Phi_nu> - sigma_mu,nu = <Phi_mu|R_nu H-bar|Phi>: E_cc on the diagonal plus
    terms from the CC residual (non-zero here because the synthetic T does not solve CC)."""
    o, v = 3, 3
    p, eri, t1, t2, _, _ = _model(o, v, 2)
    bf = fock.BruteForce(o, v, p.eps, t1, t2, eri)
    diff = bf.ip_matrix_full() - bf.ip_matrix()
    assert np.allclose(np.diag(diff)[:o], bf.e_cc(), atol=1e-12)


def test_dot_product_identity():
    o, v = 5, 6
    p = synth.make_problem(o, v, 4)
    hb = _closed(p, p.t1, p.t2)
    rng = np.random.default_rng(1)
    D = osig.dim(o, v)
    x = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    y = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    lhs = y @ osig.sigma(hb, x)
    rhs = osig.sigma_t(hb, y) @ x
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_spectral_weight_of_c_and_b():
    """With Lambda = T^dagger: c_j . b_j = 1 - sum_a (t_j^a)^2 - 1/2 sum_lab (t_jl^ab)^2."""
    o, v = 5, 7
    p = synth.make_problem(o, v, 6)
    for j in range(o):
        c = osig.c_vector(o, v, p.t1, p.t2, p.l1, p.l2, j)
        b = osig.b_vector(o, v, j)
        ref = 1.0 - np.sum(p.t1[j] ** 2) - 0.5 * np.sum(p.t2[j] ** 2)
        assert abs(c @ b - ref) < 1e-15
