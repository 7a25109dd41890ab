"""Independent literal rows (2V logit rows, one per literal: Sec. III-B's
2V x N real-valued assignment, the incomplete-assignment passage of
Sec. III-A) on the GPU against the FP64 oracle, one iteration from identical
state: every literal row normalized and binarized on its own, R counts the
literals whose own row is 1 (both rows 1: either literal satisfies its
clauses; both 0: neither does), the adjoint of a literal row sums dL/dR over
the clauses holding that literal.  Bits and histograms exact; U, g and the
AdamW outputs within the tolerances of the complete-assignment path."""
import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

from parity_util import (TOL_ADAM, TOL_GRAD, adam_bounds, adam_reference, grad_bound, make_state, oparams,
                         solver_or_skip)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    s = solver_or_skip()
    yield s
    s.close()


def mixed_cnf(V=400, seed=7):
    g = np.random.default_rng(seed)
    clauses = []
    for k in [1, 2, 3, 4, 5, 7, 9, 12] * 60:
        vs = g.choice(V - 3, size=k, replace=False) + 1
        clauses.append([int(x) * int(g.choice([-1, 1])) for x in vs])
    clauses += [[5, -5, 9], [6, 6, -8]]  # a tautology, a duplicate literal
    return gen.CNF.from_clauses(V, clauses)


def lit_one_step(solver, cnf, N, seed, t, p=None):
    p = p or tsat.default_params()
    print(f"[literal rows] V={cnf.num_vars} C={cnf.num_clauses} N={N} seed={seed} t={t} mode={p.norm_mode}",
          flush=True)
    V = cnf.num_vars
    solver.load(cnf)
    solver.set_literal_rows(True)
    th, m, v = make_state(2 * V, N, seed)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, t)
    oc = orc.Cnf.from_gen(cnf)
    hist, S, loss = solver.eval(p)
    b_ref, mu = orc.binarize(th.astype(np.float64), p.norm_mode)  # every literal row on its own
    assert np.array_equal(tsat.unpack_bits(solver.get_bits(), N), b_ref)
    H_ref = orc.lit_histogram(oc, b_ref)
    assert np.array_equal(hist.astype(np.int64), H_ref)
    S_ref, table, loss_ref = orc.smoothmin(H_ref, p.tau)
    assert np.allclose(S, S_ref, rtol=1e-12, atol=1e-12)
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-12
    U, g = solver.get_grad(p)
    U_ref = orc.lit_adjoint(oc, b_ref, table)
    aU = orc.lit_adjoint(oc, b_ref, np.abs(table))  # sum of |dL/dR| over the literal's clauses
    assert (np.abs(U - U_ref) <= TOL_GRAD * aU + 1e-30).all(), np.abs(U - U_ref).max()
    g_ref = orc.norm_backward(th.astype(np.float64), U_ref, p.norm_mode)
    ag = grad_bound(aU, th, mu, g_ref) if p.norm_mode == orc.MODE_MEAN else aU + np.abs(g_ref)
    assert (np.abs(g - g_ref) <= TOL_GRAD * ag + 1e-30).all(), np.abs(g - g_ref).max()
    rep = solver.step(1, params=p)
    assert rep.steps_done == 1
    th2, m2, v2, t2 = solver.get_state()
    assert t2 == t + 1 and th2.shape == (2 * V, N)
    th_r, m_r, v_r, lr = adam_reference(th, m, v, g, t, p)
    bt, bm, bv = adam_bounds(th, m, v, g, t, p, lr, v_r)
    assert (np.abs(m2 - m_r) <= TOL_ADAM * bm + 1e-30).all()
    assert (np.abs(v2 - v_r) <= TOL_ADAM * bv + 1e-30).all()
    assert (np.abs(th2 - th_r) <= TOL_ADAM * bt + 1e-30).all()
    b2, _ = orc.binarize(th2.astype(np.float64), p.norm_mode)
    assert np.array_equal(tsat.unpack_bits(solver.get_bits(), N), b2)
    # the oracle's own iteration over literal rows gives the same histogram
    r = orc.step(oc, th.astype(np.float64), m.astype(np.float64), v.astype(np.float64), t, p=oparams(p),
                 literal_rows=True)
    assert np.array_equal(r["H"], H_ref)


@pytest.mark.parametrize("N", [1, 64, 100, 256])
def test_literal_rows_uniform_width(solver, N):
    lit_one_step(solver, gen.planted_ksat(300, 1230, 3, seed=11), N, 5000 + N, 7)


@pytest.mark.parametrize("N", [64, 130])
def test_literal_rows_mixed_widths(solver, N):
    lit_one_step(solver, mixed_cnf(), N, 5100 + N, 40)


def test_literal_rows_none_mode(solver):
    p = tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)
    lit_one_step(solver, gen.planted_ksat(250, 1000, 3, seed=12), 96, 5200, 3, p=p)


def test_literal_rows_many_steps_stay_consistent(solver):
    """After 30 iterations (a schedule step included) the bits are still the
    binarization of the logits and the histogram that of the bits."""
    cnf = mixed_cnf(seed=9)
    solver.load(cnf)
    solver.set_literal_rows(True)
    solver.init_batch(64, seed=3)
    solver.step(30)
    th, _, _, t = solver.get_state()
    assert t == 30
    b = tsat.unpack_bits(solver.get_bits(), 64)
    b_ref, _ = orc.binarize(th.astype(np.float64))
    assert np.array_equal(b, b_ref)
    hist, _, _ = solver.eval()
    assert np.array_equal(hist.astype(np.int64), orc.lit_histogram(orc.Cnf.from_gen(cnf), b_ref))


def test_literal_rows_limits(solver):
    cnf = gen.planted_ksat(100, 410, 3, seed=13)
    solver.load(cnf)
    solver.set_literal_rows(True)
    with pytest.raises(tsat.TsatError) as e:
        solver.init_batch(300, seed=1)  # beyond the window gather's 256 candidates
    assert e.value.code == tsat.E_ARG
    solver.init_batch(64, seed=1)
    for call in (lambda: solver.get_assignment(0), lambda: solver.extract_partial(4)):
        with pytest.raises(tsat.TsatError) as e:
            call()
        assert e.value.code == tsat.E_STATE
    with pytest.raises(tsat.TsatError) as e:
        solver.set_launch_config(clause_planes=0)
    assert e.value.code == tsat.E_ARG
    solver.set_literal_rows(False)
    solver.init_batch(64, seed=1)
    assert solver.get_logits().shape == (100, 64)
    wide = gen.CNF.from_clauses(40, [list(range(1, 18))] + [[1, 2, 3]])
    solver.load(wide)
    with pytest.raises(tsat.TsatError) as e:
        solver.set_literal_rows(True)  # a clause wider than 15
    assert e.value.code == tsat.E_ARG
    solver.load_batch([cnf, cnf])
    with pytest.raises(tsat.TsatError) as e:
        solver.set_literal_rows(True)
    assert e.value.code == tsat.E_STATE
