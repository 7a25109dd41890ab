"""Batched multi-instance solving (instances of uneven size in one launch per
kernel) and graph replay, against the oracle and against single-instance runs."""
import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

from parity_util import (TOL_ADAM, TOL_GRAD, abs_adjoint, adam_bounds, adam_reference, grad_bound, make_state,
                         solver_or_skip)

pytestmark = pytest.mark.gpu

SIZES = [(120, 500, 1), (333, 1370, 2), (64, 260, 3), (1000, 4100, 4), (257, 1050, 5)]


@pytest.fixture(scope="module")
def solver():
    s = solver_or_skip()
    yield s
    s.close()


def instances(kind="planted"):
    if kind == "mixed":
        return [gen.structured(640, 3000, seed=4), gen.planted_ksat(200, 800, 3, seed=9),
                gen.structured(1280, 5000, seed=6)]
    return [gen.planted_ksat(V, C, 3, seed=s) for V, C, s in SIZES]


def stacked_state(cnfs, N, seed):
    parts = [make_state(c.num_vars, N, seed + j) for j, c in enumerate(cnfs)]
    return tuple(np.concatenate([p[k] for p in parts]) for k in range(3))


@pytest.mark.parametrize("kind,N", [("planted", 32), ("planted", 100), ("mixed", 64)])
def test_batch_one_step_parity_per_instance(solver, kind, N):
    cnfs = instances(kind)
    print(f"[batch] kind={kind} N={N} instances={len(cnfs)}", flush=True)
    solver.load_batch(cnfs)
    assert solver.num_instances == len(cnfs)
    th, m, v = stacked_state(cnfs, N, 300)
    t = 7
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, t)
    hist, S, loss = solver.eval()
    bits = tsat.unpack_bits(solver.get_bits(), N)
    U, g = solver.get_grad()
    solver.step(1)
    th2, m2, v2, _ = solver.get_state()
    bits2 = tsat.unpack_bits(solver.get_bits(), N)
    p = tsat.default_params()
    base = 0
    loss_sum = 0.0
    for j, c in enumerate(cnfs):
        r = slice(base, base + c.num_vars)
        base += c.num_vars
        oc = orc.Cnf.from_gen(c)
        b, mu = orc.binarize(th[r].astype(np.float64))
        assert np.array_equal(bits[r], b)
        H = orc.histogram(oc, b)
        K1 = hist.shape[2]
        Hp = np.zeros((N, K1), dtype=np.int64)
        Hp[:, :H.shape[1]] = H
        assert np.array_equal(hist[j].astype(np.int64), Hp), j
        S_ref, table, l_ref = orc.smoothmin(H, 1.0)
        assert np.allclose(S[j], S_ref, rtol=1e-12, atol=1e-12)
        loss_sum += l_ref
        U_ref = orc.adjoint(oc, b, table)
        aU = abs_adjoint(oc, b, table)
        assert (np.abs(U[r] - U_ref) <= TOL_GRAD * aU + 1e-30).all(), j
        g_ref = orc.norm_backward(th[r].astype(np.float64), U_ref)
        assert (np.abs(g[r] - g_ref) <= TOL_GRAD * grad_bound(aU, th[r], mu, g_ref) + 1e-30).all(), j
        th_r, m_r, v_r, lr = adam_reference(th[r], m[r], v[r], g[r], t, p)
        bt, bm, bv = adam_bounds(th[r], m[r], v[r], g[r], t, p, lr, v_r)
        assert (np.abs(th2[r] - th_r) <= TOL_ADAM * bt + 1e-30).all(), j
        b2, _ = orc.binarize(th2[r].astype(np.float64))
        assert np.array_equal(bits2[r], b2)
    assert abs(loss - loss_sum) <= 1e-9 * abs(loss_sum)


def test_batch_equals_single_instance_runs(solver):
    cnfs = instances()
    N = 64
    th, _, _ = stacked_state(cnfs, N, 400)
    solver.load_batch(cnfs)
    solver.init_batch(N, init_logits=th)
    solver.step(25)
    thb = solver.get_logits()
    base = 0
    for j, c in enumerate(cnfs):
        r = slice(base, base + c.num_vars)
        base += c.num_vars
        solver.load(c)
        solver.init_batch(N, init_logits=th[r])
        solver.step(25)
        assert np.array_equal(solver.get_logits(), thb[r]), j


@pytest.mark.parametrize("kind,N", [("planted", 32), ("mixed", 64), ("structured", 128)])
def test_graph_replay_equals_eager(solver, kind, N):
    """Replayed iterations give the eager ones bit for bit: uniform widths
    (one forward launch per bucket, the pair update at N = 32), a mixed-width
    batch (the one-launch forward with the wide histogram pass, the level
    gather with its window-filling work items) and one structured instance
    at N = 128 (the full-row instance of the level gather)."""
    cnfs = [gen.structured(2000, 9000, seed=8)] if kind == "structured" else instances(kind)
    print(f"[graph] kind={kind} N={N}", flush=True)
    th, _, _ = stacked_state(cnfs, N, 500)
    solver.load_batch(cnfs)
    outs = []
    for graph in (False, True, True):
        solver.set_graph(graph)
        solver.init_batch(N, init_logits=th)
        rep = solver.step(31)  # odd: the last iteration runs eagerly after the graph replays
        assert rep.steps_done == 31 and rep.next_step == 31
        outs.append((solver.get_logits(), solver.get_bits()))
    solver.set_graph(False)
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_freeze_on_sat_per_instance(solver):
    p = tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)
    cnfs = [gen.planted_ksat(200, 800, 3, seed=s) for s in range(1, 9)] + [gen.random_ksat(18, 130, 3, seed=13)]
    solver.load_batch(cnfs)
    N = 64
    th = np.concatenate([gen.normal_logits(c.num_vars, N, 1000 + j) for j, c in enumerate(cnfs)])
    solver.set_graph(True)
    solver.init_batch(N, init_logits=th)
    rep = solver.step(800, params=p, stop_on_sat=True)
    solver.set_graph(False)
    st = solver.instance_status()
    assert st[-1]["first_sat_step"] == -1 and st[-1]["frozen"] == 0  # unsatisfiable member
    solved = [j for j, x in enumerate(st) if x["first_sat_step"] >= 0]
    assert solved, "no tiny planted instance solved in 800 steps"
    assert rep.first_sat_step == min(st[j]["first_sat_step"] for j in solved)
    for j in solved:
        x = st[j]
        assert x["frozen"] == 1 and x["sat_ticks"] >= x["start_ticks"] > 0
        vals, cand = solver.get_witness_instance(j, cnfs[j].num_vars)
        assert cand == x["sat_candidate"]
        _, ok = orc.check(orc.Cnf.from_gen(cnfs[j]), vals[:, None])
        assert ok[0] == 1
    # a frozen instance keeps its state while the others move on
    th_a = solver.get_logits()
    solver.step(5, params=p, stop_on_sat=True)
    th_b = solver.get_logits()
    base = np.cumsum([0] + [c.num_vars for c in cnfs])
    for j in solved:
        assert np.array_equal(th_a[base[j]:base[j + 1]], th_b[base[j]:base[j + 1]])
    assert not np.array_equal(th_a[base[-2]:base[-1]], th_b[base[-2]:base[-1]])
    assert solver.device_clock_hz() > 0


def test_handoff_stop_mode_freezes_at_convergence(solver):
    """Stop mode 2 freezes each instance at its first converged (or
    satisfied) iteration, the hand-off point; frozen bits stay put."""
    cnfs = [gen.planted_ksat(300 + 40 * j, int(4.1 * (300 + 40 * j)), 3, seed=70 + j) for j in range(6)]
    solver.load_batch(cnfs)
    p = tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)
    solver.init_batch(64, seed=3)
    r = solver.step(2000, params=p, stop_on_sat=2)
    st = solver.instance_status()
    assert r.steps_done < 2000
    for x in st:
        assert x["frozen"] == 1
        first = [s for s in (x["first_sat_step"], x["first_converged_step"]) if s >= 0]
        assert first
        if x["first_converged_step"] >= 0:
            assert x["conv_ticks"] >= x["start_ticks"] > 0
            assert x["best_sat_count"] > 0.99 * x["num_clauses"]
    bits = solver.get_bits()
    solver.step(5, params=p, stop_on_sat=2)
    assert np.array_equal(solver.get_bits(), bits)


def test_ragged_witness_check_uses_the_library():
    """The ragged report verifies witnesses with the library's exact check:
    a planted assignment holds, its complement and a CNF with an empty clause
    do not (the expected verdicts come from the generator's planted
    assignment and a naive clause evaluation here)."""
    from paper_2511_07737_amd import ragged

    c = gen.planted_ksat(500, 2100, 3, seed=3)
    assert ragged.witness_holds(c, c.planted)
    flipped = (1 - c.planted).astype(np.uint8)
    naive = all(any((flipped[abs(x) - 1] == 1) == (x > 0) for x in c.clause(j)) for j in range(c.num_clauses))
    assert ragged.witness_holds(c, flipped) == naive
    assert not ragged.witness_holds(gen.CNF.from_clauses(3, [[1], []]), np.ones(3, np.uint8))
