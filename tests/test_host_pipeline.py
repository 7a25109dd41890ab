"""Host-side pieces of the ragged batch and the learned-proposal pipeline."""
import numpy as np

from paper_2511_07737_amd import gen, learned, ragged, tsat


def test_parallel_generation_matches_sequential():
    a = ragged.generate(24, seed=11, vmin=100, vmax=3000, workers=4)
    b = gen.ragged_set(24, seed=11, vmin=100, vmax=3000)
    assert all(x.num_vars == y.num_vars and np.array_equal(x.lits, y.lits) for x, y in zip(a, b))
    sizes = [c.num_vars for c in b]
    assert min(sizes) >= 100 and max(sizes) <= 3000
    ratios = [c.num_clauses / c.num_vars for c in b]
    assert 3.79 <= min(ratios) and max(ratios) <= 4.21


def test_censored_percentiles():
    # 10 instances, 4 solved: the median lies among the censored ones
    solved = [5.0, 1.0, 3.0, 2.0]
    assert ragged.censored_percentile(solved, 10, 50) is None
    assert ragged.censored_percentile(solved, 10, 10) == 1.0  # rank 1
    assert ragged.censored_percentile(solved, 10, 40) == 5.0  # rank 4
    assert ragged.censored_percentile(solved, 10, 41) is None  # rank 5
    # nothing censored: the order statistic of rank ceil(q n / 100)
    xs = np.arange(100, 0, -1).astype(float)
    assert ragged.censored_percentile(xs, 100, 50) == 50.0
    assert ragged.censored_percentile(xs, 100, 99) == 99.0
    assert ragged.censored_percentile(xs, 100, 100) == 100.0
    assert ragged.censored_percentile([], 0, 50) is None
    assert ragged.censored_percentile([], 3, 1) is None


def test_column_bits_matches_pack_helpers():
    g = np.random.default_rng(2)
    b = g.integers(0, 2, size=(50, 130)).astype(np.uint8)
    p = tsat.pack_bits(b)
    for cand in (0, 63, 64, 129):
        assert np.array_equal(learned.column_bits(p, cand), b[:, cand])


def test_corpus_and_parameter_layout():
    cs = learned.corpus(6, vmin=1000, vmax=2000, workers=2)
    assert [c.num_vars for c in cs] == [c.num_vars for c in learned.corpus(6, vmin=1000, vmax=2000, workers=1)]
    for c in cs:
        assert 1000 <= c.num_vars <= 2000 and abs(c.num_clauses - 4.1 * c.num_vars) <= 1
    p = learned.init_params(3)
    assert p.shape == (tsat.MLP_NUM_PARAMS,) and p.dtype == np.float32
    assert sum(int(np.prod(s)) for _, s in learned.SHAPES) == tsat.MLP_NUM_PARAMS


def test_weights_roundtrip(tmp_path):
    p = learned.init_params(4)
    path = str(tmp_path / "w" / "m.npz")
    learned.save_weights(path, p, {"a": 1})
    q, meta = learned.load_weights(path)
    assert np.array_equal(p, q) and meta == {"a": 1}


def test_majority_proposal_counts_polarities():
    # variable 1: +,+,- ; variable 2: -,- ; variable 3: never occurs
    a = gen.CNF.from_clauses(3, [[1, -2], [1, -2], [-1]])
    b = gen.CNF.from_clauses(2, [[2], [-1, 2]])
    p = learned.majority_proposal([a, b])
    assert p.dtype == np.float32 and p.shape == (5,)
    expect = [(2 + 1) / (3 + 2), (0 + 1) / (2 + 2), 0.5, (0 + 1) / (1 + 2), (2 + 1) / (2 + 2)]
    assert np.allclose(p, expect)
    # the most likely value is the majority vote; it agrees with a planted
    # 3-SAT assignment on about 70% of the variables at ratio 4.1
    c = gen.planted_ksat(4000, 16400, 3, seed=5)
    agree = ((learned.majority_proposal(c) > 0.5) == (c.planted > 0)).mean()
    assert 0.6 < agree < 0.8
