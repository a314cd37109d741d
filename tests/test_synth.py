"""The seeded input generator: symmetry, moments, determinism, block consistency."""
import numpy as np

import synth


def test_antisymmetry_and_hermiticity():
    p = synth.make_problem(3, 4, 7)
    g = p.full_eri()
    assert np.array_equal(g, -g.transpose(1, 0, 2, 3))
    assert np.array_equal(g, -g.transpose(0, 1, 3, 2))
    assert np.array_equal(g, g.transpose(2, 3, 0, 1))


def test_blocks_are_slices_of_one_tensor():
    o, v = 3, 4
    p = synth.make_problem(o, v, 2)
    g = p.full_eri()
    O, V = slice(0, o), slice(o, o + v)
    for kind in ("oooo", "ooov", "oovv", "ovvo", "ovvv"):
        sl = tuple(O if c == "o" else V for c in kind)
        assert np.array_equal(p.block(kind), g[sl]), kind


def test_moments_and_determinism():
    a = synth.eri_block(11, 8, 40, "ovvv")
    b = synth.eri_block(11, 8, 40, "ovvv")
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.eri_block(12, 8, 40, "ovvv"))
    off = a[a != 0]
    assert abs(off.std() - 0.05) < 0.002
    assert abs(off.mean()) < 0.001
    t1 = synth.normal(3, synth.STREAM_T1, 20000, 0.01)
    assert abs(t1.std() - 0.01) < 3e-4


def test_orbital_energies_and_t2():
    p = synth.make_problem(10, 20, 0)
    eo, ev = p.eps[:10], p.eps[10:]
    assert np.all(np.diff(eo) >= 0) and np.all(np.diff(ev) >= 0)
    assert eo.min() >= -1.5 and eo.max() <= -0.3 and ev.min() >= 0.1 and ev.max() <= 2.0
    i, j, a, b = 1, 4, 3, 7
    den = eo[i] + eo[j] - ev[a] - ev[b]
    assert np.isclose(p.t2[i, j, a, b], p.block("oovv")[i, j, a, b] / den, rtol=0, atol=1e-16)
    assert np.array_equal(p.l2, p.t2) and np.array_equal(p.l1, p.t1)
