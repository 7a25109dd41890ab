"""Pins of the oracle's two variants of the method (CPU only):

* assignment mixing at a learning-rate restart (Sec. IV-A, the paragraph the
  source leaves commented out, and its equation), with the optimizer reset;
* independent literal rows (A_real with 2V rows, Sec. III-B; the
  incomplete-assignment passage of Sec. III-A, commented out in the source).

Each pin checks the oracle against something other than itself: brute-force
enumeration with a naive clause evaluation, closed forms, reductions to the
already pinned complete-assignment functions, finite differences of a
relaxed objective written here in numpy, and torch.optim.AdamW.
"""
import itertools

import numpy as np
import pytest

from paper_2511_07737_amd import gen


def _naive_sat_counts(clauses, vals):
    """Satisfied clauses of a complete 0/1 assignment vals[V] (set semantics)."""
    true_lits = {v + 1 if vals[v] else -(v + 1) for v in range(len(vals))}
    return sum(1 for c in clauses if true_lits & set(c))


# ------------------------------------------------------------------ mixing


def test_mix_keeps_the_best_column_and_averages_the_rest(orc):
    rng = np.random.default_rng(1)
    th = rng.standard_normal((7, 9))
    for istar in (0, 4, 8):
        out = orc.mix(th, istar)
        assert np.array_equal(out[:, istar], th[:, istar])
        others = [i for i in range(9) if i != istar]
        # distances to the best column halve
        d0 = np.abs(th[:, others] - th[:, [istar]])
        d1 = np.abs(out[:, others] - out[:, [istar]])
        assert np.allclose(d1, 0.5 * d0, rtol=1e-15, atol=1e-15)
        # closed form of the new row mean: (old mean + best entry) / 2
        assert np.allclose(out.mean(axis=1), 0.5 * (th.mean(axis=1) + th[:, istar]), rtol=1e-14, atol=1e-15)
        # entries that agree in sign with the best one keep that sign
        agree = np.sign(th) == np.sign(th[:, [istar]])
        assert (np.sign(out)[agree] == np.sign(th)[agree]).all()


def test_mix_fixed_point_and_composition(orc):
    rng = np.random.default_rng(2)
    col = rng.standard_normal((5, 1))
    same = np.repeat(col, 6, axis=1)
    assert np.array_equal(orc.mix(same, 3), same)
    th = rng.standard_normal((5, 6))
    twice = orc.mix(orc.mix(th, 2), 2)
    assert np.allclose(twice, 0.25 * th + 0.75 * th[:, [2]], rtol=1e-15, atol=1e-15)
    with pytest.raises(ValueError):
        orc.mix(th, 6)


def test_best_candidate_by_enumeration(orc):
    cnf = gen.planted_ksat(12, 50, 3, seed=7)
    oc = orc.Cnf.from_gen(cnf)
    clauses = [list(cnf.clause(c)) for c in range(cnf.num_clauses)]
    rng = np.random.default_rng(3)
    for trial in range(20):
        b = rng.integers(0, 2, size=(12, 16)).astype(np.uint8)
        if trial % 4 == 0:
            b[:, 9] = b[:, 2]  # a tie between two columns
        sat = [_naive_sat_counts(clauses, b[:, i]) for i in range(16)]
        want = int(np.argmax(sat))  # first maximum: the lower index on ties
        assert orc.best_candidate(orc.histogram(oc, b)) == want


def test_mixing_iteration_schedule_and_optimizer_reset(orc):
    torch = pytest.importorskip("torch")
    cnf = gen.planted_ksat(200, 800, 3, seed=1)
    oc = orc.Cnf.from_gen(cnf)
    rng = np.random.default_rng(4)
    th = rng.standard_normal((200, 32))
    m = 0.05 * rng.standard_normal((200, 32))
    v = 0.01 * np.abs(rng.standard_normal((200, 32))) + 1e-6
    for mode in (orc.MODE_MEAN, orc.MODE_NONE):
        pm = orc.default_params(mix=1, mode=mode, tau=2.0)
        p0 = orc.default_params(mix=0, mode=mode, tau=2.0)
        # not a restart iteration: identical to the method without mixing
        for t in (0, 359, 361, 719):
            a, b = orc.step(oc, th, m, v, t, pm), orc.step(oc, th, m, v, t, p0)
            assert a["mixed"] == -1 and np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["m"], b["m"])
        # a restart iteration: mix into the best candidate of this forward
        # pass, moments to zero, no gradient step
        for t in (360, 720):
            r = orc.step(oc, th, m, v, t, pm)
            istar = orc.best_candidate(r["H"])
            assert r["mixed"] == istar
            assert np.array_equal(r["theta"], orc.mix(th, istar))
            assert not r["m"].any() and not r["v"].any() and not r["g"].any()
            assert np.array_equal(r["bits"], orc.binarize(th, mode)[0])
        # the next update is the first step of a fresh AdamW on the mixed logits
        r = orc.step(oc, th, m, v, 360, pm)
        nxt = orc.step(oc, r["theta"], r["m"], r["v"], 361, pm, t_reset=361)
        T = torch.tensor(r["theta"], dtype=torch.float64, requires_grad=True)
        opt = torch.optim.AdamW([T], lr=orc.lr(361), betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-2)
        T.grad = torch.tensor(nxt["g"], dtype=torch.float64)
        opt.step()
        assert np.allclose(nxt["theta"], T.detach().numpy(), rtol=1e-12, atol=1e-14)
        # without the reset (the method's own restart), the moments carry on
        cont = orc.step(oc, th, m, v, 360, p0)
        assert cont["mixed"] == -1 and cont["m"].any()


# ----------------------------------------------------- independent literal rows


def _lit_rows(clause_lits):
    return [2 * (abs(x) - 1) + (0 if x > 0 else 1) for x in clause_lits]


def test_literal_rows_brute_force_dont_care(orc):
    """Every assignment of both literal rows of 4 variables (4^4 candidates):
    R counts the literals whose own row is 1; both rows 1 ("don't care")
    satisfies every clause holding either literal, both 0 none."""
    clauses = [[1, -2, 3], [-1, 4], [2, 3, -4], [-3], [1, -1, 2], [4, -2, -3, 1]]
    cnf = gen.CNF.from_clauses(4, clauses)
    oc = orc.Cnf.from_gen(cnf)
    cands = list(itertools.product((0, 1), repeat=8))  # (row 0, row 1, ..., row 7)
    N = len(cands)
    bl = np.array(cands, dtype=np.uint8).T.copy()  # [2V][N]
    H = orc.lit_histogram(oc, bl)
    K = max(len(set(c)) for c in clauses)
    for i, cand in enumerate(cands):
        want = np.zeros(K + 1, dtype=np.int64)
        for c in clauses:
            want[sum(cand[r] for r in set(_lit_rows(c)))] += 1
        assert np.array_equal(H[i], want), i
        sat_all = all(any(cand[r] for r in _lit_rows(c)) for c in clauses)
        assert (H[i, 0] == 0) == sat_all
    dc = cands.index((1,) * 8)
    none = cands.index((0,) * 8)
    assert H[dc, 0] == 0 and H[none, 0] == len(clauses)


def test_literal_rows_reduce_to_complete_assignments(orc):
    cnf = gen.structured(2000, 6000, seed=5)
    oc = orc.Cnf.from_gen(cnf)
    rng = np.random.default_rng(6)
    b = rng.integers(0, 2, size=(2000, 40)).astype(np.uint8)
    bl = np.empty((4000, 40), dtype=np.uint8)
    bl[0::2], bl[1::2] = b, 1 - b
    H = orc.histogram(oc, b)
    assert np.array_equal(orc.lit_histogram(oc, bl), H)
    _, table, _ = orc.smoothmin(H, 1.5)
    U2 = orc.lit_adjoint(oc, bl, table)
    U = orc.adjoint(oc, b, table)
    assert np.allclose(U2[0::2] - U2[1::2], U, rtol=1e-12, atol=1e-13)


def _relaxed_lit_S(clause_rows, x, i, tau):
    """SmoothMin (Eq. 4) of R~_c = sum over the literals of c of x[row][i]."""
    R = np.array([x[rows, i].sum() for rows in clause_rows])
    w = np.exp(-tau * (R - R.min()))
    return float((R * w).sum() / w.sum())


def test_literal_adjoint_finite_differences(orc):
    cnf = gen.planted_ksat(30, 120, 3, seed=9)
    oc = orc.Cnf.from_gen(cnf)
    clause_rows = [np.array(_lit_rows(cnf.clause(c))) for c in range(cnf.num_clauses)]
    rng = np.random.default_rng(10)
    N, tau, h = 6, 1.0, 1e-4
    bl = rng.integers(0, 2, size=(60, N)).astype(np.uint8)
    w = rng.standard_normal(N)
    H = orc.lit_histogram(oc, bl)
    _, table, _ = orc.smoothmin(H, tau, w)
    U2 = orc.lit_adjoint(oc, bl, table)
    x = bl.astype(np.float64)
    for row, i in zip(rng.integers(0, 60, 40), rng.integers(0, N, 40)):
        xp, xm = x.copy(), x.copy()
        xp[row, i] += h
        xm[row, i] -= h
        fd = w[i] * (_relaxed_lit_S(clause_rows, xp, i, tau) - _relaxed_lit_S(clause_rows, xm, i, tau)) / (2 * h)
        assert abs(fd - U2[row, i]) <= 1e-6 * (1 + abs(U2[row, i])), (row, i, fd, U2[row, i])


def test_literal_row_step_uses_per_literal_normalization(orc):
    """The literal-row iteration: Eq. 5 and Eq. 2 per literal row, the
    literal histogram, the literal adjoint, Eq. 5's backward per row."""
    cnf = gen.planted_ksat(100, 410, 3, seed=11)
    oc = orc.Cnf.from_gen(cnf)
    rng = np.random.default_rng(12)
    th = rng.standard_normal((200, 16))
    z = np.zeros_like(th)
    for mode in (orc.MODE_MEAN, orc.MODE_NONE):
        p = orc.default_params(mode=mode)
        r = orc.step(oc, th, z, z, 0, p, literal_rows=True)
        bl, _ = orc.binarize(th, mode)
        assert np.array_equal(r["bits"], bl)
        H = orc.lit_histogram(oc, bl)
        assert np.array_equal(r["H"], H)
        _, table, loss = orc.smoothmin(H, 1.0)
        assert r["loss"] == pytest.approx(loss, rel=1e-14)
        U2 = orc.lit_adjoint(oc, bl, table)
        assert np.allclose(r["g"], orc.norm_backward(th, U2, mode), rtol=1e-13, atol=1e-15)
        # rows of both literals of a variable are independent: the x_v and
        # not-x_v rows can both be 1 at once
        assert ((r["bits"][0::2] == 1) & (r["bits"][1::2] == 1)).any()
