"""GPU (gfx950) path vs the FP64 oracle, one iteration from identical state.

Every GPU value comes through the C-ABI (``paper_2511_07737_amd.tsat``).
Inputs are seeded and synthetic; expected values come only from ``oracle``.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

from parity_util import (TOL_ADAM, TOL_GRAD, abs_adjoint, adam_bounds, adam_reference, grad_bound,
                         make_state, one_step_parity, oparams, solver_or_skip, sub_cnf)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    s = solver_or_skip()
    yield s
    s.close()


def test_tiny_first_step(solver):
    cnf = gen.planted_ksat(200, 800, 3, seed=1)
    th, _, _ = make_state(200, 64, 1001, t_moments=False)
    one_step_parity(solver, cnf, 64, 1001, 0, state=(th, np.zeros_like(th), np.zeros_like(th)))


@pytest.mark.parametrize("t", [37, 335, 361])
def test_tiny_mid_schedule(solver, t):
    cnf = gen.planted_ksat(200, 800, 3, seed=2)
    one_step_parity(solver, cnf, 64, 1002 + t, t)


@pytest.mark.parametrize("N", [1, 63, 100, 130, 256])
def test_ragged_candidate_counts(solver, N):
    cnf = gen.planted_ksat(300, 1230, 3, seed=3)
    one_step_parity(solver, cnf, N, 2000 + N, 5)


def mixed_edge_cnf():
    s = gen.structured(640, 3000, seed=4)
    clauses = [list(s.clause(c)) for c in range(s.num_clauses)]
    # duplicate literals, tautologies, unit clauses; variables 641..650 never occur
    clauses += [[5, 5, -7], [9, -9], [11, -11, 12], [13], [-14], [15, 16, 15, -16]]
    return gen.CNF.from_clauses(650, clauses)


def test_mixed_widths_and_edge_clauses(solver):
    one_step_parity(solver, mixed_edge_cnf(), 130, 31, 12)


def very_wide_cnf():
    """Clauses of every width 5..32 (the widest the store takes), so each
    width class of the wide-clause forward runs, next to some 3-clauses."""
    rng = np.random.default_rng(17)
    V = 400
    clauses = []
    for k in range(5, 33):
        for _ in range(40):
            vs = rng.choice(V, size=k, replace=False) + 1
            clauses.append([int(x) for x in vs * rng.choice([-1, 1], size=k)])
    for _ in range(600):
        vs = rng.choice(V, size=3, replace=False) + 1
        clauses.append([int(x) for x in vs * rng.choice([-1, 1], size=3)])
    return gen.CNF.from_clauses(V, clauses)


@pytest.mark.parametrize("N", [100, 32])
def test_very_wide_clauses(solver, N):
    one_step_parity(solver, very_wide_cnf(), N, 41, 3)


def heavy_cnf():
    """Mixed widths where two variables occur in thousands of clauses: their
    occurrence records are split into chunks summed by separate waves."""
    g = np.random.default_rng(17)
    clauses = []
    for _ in range(2500):
        k = int(g.integers(2, 7))
        vs = g.choice(np.arange(3, 401), size=k, replace=False)
        clauses.append([int(v) if g.random() < 0.5 else -int(v) for v in vs])
    for hv, n in ((1, 1500), (2, 300)):
        for _ in range(n):
            k = int(g.integers(1, 6))
            vs = g.choice(np.arange(3, 401), size=k, replace=False)
            cl = [int(v) if g.random() < 0.5 else -int(v) for v in vs]
            cl.append(hv if g.random() < 0.5 else -hv)
            clauses.append(cl)
    return gen.CNF.from_clauses(400, clauses)


@pytest.mark.parametrize("mode", [tsat.MODE_MEAN, tsat.MODE_NONE])
def test_heavy_variables_split_into_chunks(solver, mode):
    one_step_parity(solver, heavy_cnf(), 100, 61, 5, p=tsat.default_params(norm_mode=mode))


def test_none_mode(solver):
    p = tsat.default_params(norm_mode=tsat.MODE_NONE)
    one_step_parity(solver, gen.planted_ksat(200, 800, 3, seed=5), 64, 41, 3, p=p)


@pytest.mark.parametrize("tau", [0.0, 0.5, 2.0])
def test_temperatures(solver, tau):
    p = tsat.default_params(tau=tau)
    one_step_parity(solver, gen.planted_ksat(150, 600, 3, seed=6), 96, 51, 9, p=p)


def test_zero_mean_row_uses_clamp(solver):
    cnf = gen.planted_ksat(50, 200, 3, seed=7)
    th, m, v = make_state(50, 64, 61)
    th[3] = np.tile(np.array([1.5, -1.5, 0.25, -0.25], dtype=np.float32), 16)  # mean exactly 0
    _, mu = orc.binarize(th.astype(np.float64))
    assert mu[3] == 1e-12
    out = one_step_parity(solver, cnf, 64, 61, 4, state=(th, m, v))
    assert np.abs(out["g"][3]).max() > 1e6  # U / 1e-12


def test_empty_clause_never_sat(solver):
    cnf = gen.CNF.from_clauses(20, [[1, 2], [], [-3, 4, 5]])
    one_step_parity(solver, cnf, 64, 71, 0)
    sat, ok = solver.check()
    assert ok.sum() == 0 and (sat <= 2).all()


def test_no_clauses_everything_sat(solver):
    cnf = gen.CNF.from_clauses(5, [])
    solver.load(cnf)
    solver.init_batch(10, seed=3)
    sat, ok = solver.check()
    assert ok.all() and (sat == 0).all()
    hist, S, loss = solver.eval()
    assert (S == 0).all() and loss == 0.0


# ---------------------------------------------------------------------------
# full-size configurations, sampled outputs (launch configuration of the bench)
# ---------------------------------------------------------------------------

def sampled_parity(solver, cnf, N, seed, t, nsample=48, full_hist=True):
    p = tsat.default_params()
    print(f"[sampled] V={cnf.num_vars} C={cnf.num_clauses} N={N} t={t}", flush=True)
    solver.load(cnf)
    th, m, v = make_state(cnf.num_vars, N, seed)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, t)
    oc = orc.Cnf.from_gen(cnf)
    b_ref, mu = orc.binarize(th.astype(np.float64))
    assert np.array_equal(tsat.unpack_bits(solver.get_bits(), N), b_ref)
    hist, S, loss = solver.eval(p)
    H_ref = orc.histogram(oc, b_ref)
    assert np.array_equal(hist.astype(np.int64), H_ref)
    S_ref, table, loss_ref = orc.smoothmin(H_ref, p.tau)
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref)
    U_gpu, g_gpu = solver.get_grad(p)
    rng = np.random.default_rng(seed)
    deg = np.bincount(np.abs(cnf.lits) - 1, minlength=cnf.num_vars)
    pick = np.unique(np.concatenate([rng.choice(cnf.num_vars, nsample, replace=False),
                                     np.argsort(deg)[-4:]]))  # include the highest-degree variables
    sub = sub_cnf(cnf, pick)
    osub = orc.Cnf.from_gen(sub)
    U_ref = orc.adjoint(osub, b_ref, table)[pick]
    aU_full = abs_adjoint(osub, b_ref, table)
    aU = aU_full[pick]
    assert (np.abs(U_gpu[pick] - U_ref) <= TOL_GRAD * aU + 1e-30).all()
    g_ref = orc.norm_backward(th[pick].astype(np.float64), U_ref)
    ag = grad_bound(aU, th[pick], mu[pick], g_ref)
    assert (np.abs(g_gpu[pick] - g_ref) <= TOL_GRAD * ag + 1e-30).all()
    rep = solver.step(1, params=p)
    assert rep.steps_done == 1
    th2, m2, v2, _ = solver.get_state()
    th_r, m_r, v_r, lr = adam_reference(th[pick], m[pick], v[pick], g_gpu[pick], t, p)
    bt, bm, bv = adam_bounds(th[pick], m[pick], v[pick], g_gpu[pick], t, p, lr, v_r)
    assert (np.abs(th2[pick] - th_r) <= TOL_ADAM * bt + 1e-30).all()
    assert (np.abs(m2[pick] - m_r) <= TOL_ADAM * bm + 1e-30).all()
    b2_ref, _ = orc.binarize(th2.astype(np.float64))
    assert np.array_equal(tsat.unpack_bits(solver.get_bits(), N), b2_ref)


@pytest.mark.timeout(600)
def test_large_config_sampled(solver):
    cnf = gen.planted_ksat(1_000_000, 4_100_000, 3, seed=1)
    sampled_parity(solver, cnf, 256, 1001, 0)


@pytest.mark.timeout(600)
def test_structured_config_sampled(solver):
    cnf = gen.structured(500_000, 2_500_000, seed=2)
    sampled_parity(solver, cnf, 128, 1002, 100)


# ---------------------------------------------------------------------------
# exact check, handoff, witness, method-level behaviour
# ---------------------------------------------------------------------------

def test_check_bits_brute_force(solver):
    for n, m, seed, planted in [(16, 68, 1, True), (16, 100, 2, False), (20, 85, 3, True)]:
        cnf = gen.planted_ksat(n, m, 3, seed) if planted else gen.random_ksat(n, m, 3, seed)
        print(f"[check_bits] n={n} m={m} seed={seed}", flush=True)
        solver.load(cnf)
        packed = gen.enumerate_assignments(n)
        sat, ok = solver.check_bits(packed, 1 << n)
        b = tsat.unpack_bits(packed, 1 << n)
        oc = orc.Cnf.from_gen(cnf)
        sat_ref, ok_ref = orc.check(oc, b)
        assert np.array_equal(sat, sat_ref) and np.array_equal(ok, ok_ref)
        if planted:
            zi = int(sum(int(cnf.planted[v]) << v for v in range(n)))
            assert ok[zi] == 1


def test_extract_partial_valid_selection(solver):
    cnf = mixed_edge_cnf()
    N = 64
    solver.load(cnf)
    th, m, v = make_state(cnf.num_vars, N, 91)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, 3)
    oc = orc.Cnf.from_gen(cnf)
    b, mu = orc.binarize(th.astype(np.float64))
    H = orc.histogram(oc, b)
    _, table, _ = orc.smoothmin(H, 1.0)
    U = orc.adjoint(oc, b, table)
    g = orc.norm_backward(th.astype(np.float64), U)
    ag = grad_bound(abs_adjoint(oc, b, table), th, mu, g)
    sat_ref, _ = orc.check(oc, b)
    k = 20
    ids, lits, sat = solver.extract_partial(10, k)
    order = np.lexsort((np.arange(N), -sat_ref))
    assert list(ids) == list(order[:10])
    assert np.array_equal(sat, sat_ref[ids])
    occurs = np.zeros(cnf.num_vars, bool)
    occurs[np.abs(cnf.lits) - 1] = True
    for a, i in enumerate(ids):
        sel = np.abs(lits[a]) - 1
        assert len(set(sel)) == k and occurs[sel].all()
        # the sign is the candidate's current value
        assert np.array_equal(lits[a] > 0, b[sel, i] == 1)
        # any valid choice of the k smallest |g| (ties within the gradient tolerance)
        mags = np.abs(g[:, i])
        kth = np.sort(mags[occurs])[k - 1]
        assert (mags[sel] <= kth + TOL_GRAD * ag[sel, i] + 1e-30).all()
        # most confident first
        assert (np.diff(mags[sel]) >= -TOL_GRAD * (ag[sel[1:], i] + ag[sel[:-1], i])).all()


def test_extract_partial_more_slots_than_variables(solver):
    cnf = gen.CNF.from_clauses(6, [[1, -2], [2, 3], [-1, 4]])  # 5 and 6 never occur
    solver.load(cnf)
    solver.init_batch(8, seed=5)
    ids, lits, sat = solver.extract_partial(8, 6)
    assert (lits[:, 4:] == 0).all()
    assert all(sorted(np.abs(r[:4])) == [1, 2, 3, 4] for r in lits)


def test_witness_and_stop_on_sat(solver):
    # Eq. 5 read literally pulls the batch to a per-variable consensus that
    # stalls short of all-SAT; the un-normalized mode solves this size.
    p = tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)
    cnf = gen.planted_ksat(200, 800, 3, seed=1)
    oc = orc.Cnf.from_gen(cnf)
    solver.load(cnf)
    rep = None
    for init_seed in range(1001, 1009):
        th0 = gen.normal_logits(200, 64, init_seed)
        solver.init_batch(64, init_logits=th0)
        rep = solver.step(800, params=p, stop_on_sat=True)
        if rep.first_sat_step >= 0:
            break
    assert rep.first_sat_step >= 0, "tiny planted instance not solved from 8 seeded batches"
    assert rep.steps_done == rep.first_sat_step
    vals, cand = solver.get_witness()
    _, ok = orc.check(oc, vals[:, None])
    assert ok[0] == 1 and cand == rep.sat_candidate
    # the stopped batch still holds the satisfying candidate
    assert np.array_equal(solver.get_assignment(cand), vals)
    # without stopping, the update kernel records the witness of that step
    solver.init_batch(64, init_logits=th0)
    rep2 = solver.step(rep.first_sat_step + 5, params=p, stop_on_sat=False)
    assert rep2.first_sat_step == rep.first_sat_step and rep2.steps_done == rep.first_sat_step + 5
    vals2, cand2 = solver.get_witness()
    assert np.array_equal(vals2, vals) and cand2 == cand


def test_unsat_instance_never_reports_sat(solver):
    cnf = gen.random_ksat(18, 130, 3, seed=13)
    solver.load(cnf)
    _, ok = solver.check_bits(gen.enumerate_assignments(18), 1 << 18)
    assert ok.sum() == 0, "instance is satisfiable; pick another seed"
    solver.init_batch(128, seed=99)
    rep = solver.step(400, stop_on_sat=True)
    assert rep.first_sat_step == -1 and rep.sat_candidate == -1
    sat, ok = solver.check()
    assert ok.sum() == 0


def test_deterministic_and_seeded_init(solver):
    cnf = gen.planted_ksat(2000, 8200, 3, seed=17)
    solver.load(cnf)
    outs = []
    for _ in range(2):
        solver.init_batch(128, seed=1234)
        solver.step(25)
        outs.append(solver.get_state())
    assert all(np.array_equal(a, b) for a, b in zip(outs[0][:3], outs[1][:3]))
    solver.init_batch(256, seed=77)
    th = solver.get_logits()
    assert abs(th.mean()) < 0.01 and abs(th.std() - 1.0) < 0.01
    b = tsat.unpack_bits(solver.get_bits(), 256)
    b_ref, _ = orc.binarize(th.astype(np.float64))
    assert np.array_equal(b, b_ref)
    solver.init_batch(256, seed=78)
    assert not np.array_equal(solver.get_logits(), th)


def test_error_paths(solver):
    cnf = gen.planted_ksat(30, 120, 3, seed=19)
    s2 = tsat.Solver()
    with pytest.raises(tsat.TsatError) as e:
        s2.init_batch(8)
    assert e.value.code == tsat.E_STATE
    s2.load(cnf)
    with pytest.raises(tsat.TsatError) as e:
        s2.step(1)
    assert e.value.code == tsat.E_STATE
    for n in (0, tsat.MAX_STEP_N + 1):
        with pytest.raises(tsat.TsatError) as e:
            s2.init_batch(n)
        assert e.value.code == tsat.E_ARG
    s2.init_batch(8, seed=1)
    with pytest.raises(tsat.TsatError) as e:
        s2.get_witness()
    assert e.value.code == tsat.E_STATE
    with pytest.raises(tsat.TsatError) as e:
        s2.extract_partial(9)
    assert e.value.code == tsat.E_ARG
    with pytest.raises(tsat.TsatError) as e:
        s2.step(1, params=tsat.default_params(decay_every=0))
    assert e.value.code == tsat.E_ARG
    # a NaN logit is reported as a numeric error, with the report filled
    th = s2.get_logits()
    th[0, 0] = np.nan
    s2.set_logits(th)
    with pytest.raises(tsat.TsatError) as e:
        s2.step(1)
    assert e.value.code == tsat.E_NUMERIC
    rep = s2.step(1, raise_numeric=False)
    assert rep.nonfinite == 1
    s2.close()


def test_oom_injection_subprocess(solver):
    import os
    import subprocess
    import sys

    code = (
        "import sys; sys.path.insert(0, '.');"
        "from paper_2511_07737_amd import gen, tsat;"
        "s = tsat.Solver();"
        "c = gen.planted_ksat(30, 120, 3, 1)\n"
        "try:\n    s.load(c); s.init_batch(8)\nexcept tsat.TsatError as e:\n    print('CODE', e.code)\n"
    )
    env = dict(os.environ, TSAT_FAIL_ALLOC_AFTER="4")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=120)
    assert "CODE -3" in r.stdout, r.stdout + r.stderr
