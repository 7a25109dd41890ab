"""Properties of the seeded input generators (shapes, structure, determinism)."""
import numpy as np

from paper_2511_07737_amd import gen


def test_planted_properties_and_determinism():
    a = gen.planted_ksat(500, 2050, 3, seed=4)
    b = gen.planted_ksat(500, 2050, 3, seed=4)
    assert np.array_equal(a.lits, b.lits) and np.array_equal(a.planted, b.planted)
    assert a.num_clauses == 2050 and a.num_lits == 3 * 2050
    cl = np.abs(a.lits.reshape(-1, 3))
    assert (np.sort(cl, axis=1)[:, 1:] != np.sort(cl, axis=1)[:, :-1]).all()  # distinct variables
    assert cl.min() >= 1 and cl.max() <= 500
    z = a.planted
    lit = a.lits.reshape(-1, 3)
    true = np.where(lit > 0, z[np.abs(lit) - 1] == 1, z[np.abs(lit) - 1] == 0)
    assert true.any(axis=1).all()
    # resampling until satisfied: each literal agrees with z with probability 4/7
    assert abs(true.mean() - 4 / 7) < 0.02
    assert abs((lit > 0).mean() - 0.5) < 0.02


def test_dimacs_stream_roundtrip():
    a = gen.structured(400, 1500, seed=1)
    s = a.dimacs_stream()
    assert s.size == a.num_lits + a.num_clauses and (s == 0).sum() == a.num_clauses
    ends = np.nonzero(s == 0)[0]
    assert np.array_equal(ends - np.arange(a.num_clauses), a.offsets[1:])
    text = a.to_dimacs()
    assert text.startswith("p cnf 400 1500\n")


def test_structured_shape():
    s = gen.structured(64 * 200, 40000, seed=2)
    w = s.widths()
    ks, pk = gen.width_pmf()
    freq = np.bincount(w, minlength=13)[2:13] / w.size
    assert np.allclose(freq, pk, atol=0.01)
    assert abs(w.mean() - (ks * pk).sum()) < 0.05
    v = np.abs(s.lits) - 1
    deg = np.bincount(v, minlength=s.num_vars)
    assert deg.max() > 20 * deg.mean()  # heavy-tailed occurrences
    # literals mostly stay in the clause's home community (90% of slots)
    comm = v // 200
    first = np.repeat(comm[s.offsets[:-1]], w)
    assert (comm == first).mean() > 0.75
    for c in range(0, s.num_clauses, 997):
        x = np.abs(s.clause(c))
        assert np.unique(x).size == x.size


def test_ragged_sizes():
    r = gen.ragged_set(count=40, seed=3000)
    Vs = np.array([c.num_vars for c in r])
    ratios = np.array([c.num_clauses / c.num_vars for c in r])
    assert Vs.min() >= 1000 and Vs.max() <= 200000
    assert ratios.min() >= 3.79 and ratios.max() <= 4.21
    assert len({c.num_vars for c in r}) > 30


def test_enumerate_assignments_bits():
    b = gen.enumerate_assignments(7)
    assert b.shape == (7, 2)
    for i in range(128):
        for v in range(7):
            assert (int(b[v, i // 64]) >> (i % 64)) & 1 == (i >> v) & 1
    logits = gen.normal_logits(100, 32, 9)
    assert logits.dtype == np.float32 and logits.shape == (100, 32)
    assert abs(logits.mean()) < 0.05 and abs(logits.std() - 1) < 0.05
