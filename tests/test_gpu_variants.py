"""GPU (gfx950) path vs the FP64 oracle for the method's variants:

* assignment mixing at learning-rate restarts (the mixing paragraph of
  Sec. IV-A and its equation, read as in the oracle: after the forward pass
  of an iteration t > 0 with t mod 360 = 0, every candidate other than the
  best one is averaged with it, the optimizer restarts from zero and the
  iteration takes no gradient step).

Every GPU value comes through the C-ABI; expected values come only from
``oracle``.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

from parity_util import TOL_ADAM, adam_bounds, adam_reference, make_state, solver_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    s = solver_or_skip()
    yield s
    s.close()


def oparams(p, **kw):
    return orc.default_params(tau=p.tau, lr0=p.lr0, decay=p.lr_decay, lr_min=p.lr_min, beta1=p.beta1,
                              beta2=p.beta2, eps=p.eps, weight_decay=p.weight_decay, every=p.decay_every,
                              restart=p.restart_every, mode=p.norm_mode, **kw)


def mixed_widths_cnf():
    s = gen.structured(700, 3000, seed=9)
    clauses = [list(s.clause(c)) for c in range(s.num_clauses)] + [[4, 4, -6], [8, -8], [12]]
    return gen.CNF.from_clauses(705, clauses)


CASES = {
    "planted3": lambda: gen.planted_ksat(400, 1640, 3, seed=21),   # clause-plane window gather
    "planted2": lambda: gen.planted_ksat(300, 600, 2, seed=22),    # width-2 window gather
    "mixed": mixed_widths_cnf,                                      # generic records
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("N", [64, 100])
@pytest.mark.parametrize("mode", [tsat.MODE_MEAN, tsat.MODE_NONE])
def test_mixing_at_restart_and_next_update(solver, case, N, mode):
    """Iteration 360 with mixing on: the forward as usual, then theta mixed
    into the best candidate (bit-exact against the oracle's FP64 average
    rounded to FP32), m = v = 0, new bits exact, no gradient step; iteration
    361 is the first step of a fresh AdamW (bias-correction count 1)."""
    cnf = CASES[case]()
    print(f"[mix] case={case} N={N} mode={mode}", flush=True)
    solver.load(cnf)
    oc = orc.Cnf.from_gen(cnf)
    th, m, v = make_state(cnf.num_vars, N, 4000 + N)
    p = tsat.default_params(norm_mode=mode, mix=1)
    op = oparams(p, mix=1)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, 360)
    ref = orc.step(oc, th.astype(np.float64), m.astype(np.float64), v.astype(np.float64), 360, op)
    assert ref["mixed"] >= 0
    rep = solver.step(1, params=p)
    assert rep.steps_done == 1 and rep.next_step == 361
    assert rep.best_candidate == ref["mixed"]
    assert abs(rep.loss - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    th1, m1, v1, t1 = solver.get_state()
    assert t1 == 361
    assert np.array_equal(th1, ref["theta"].astype(np.float32))
    assert not m1.any() and not v1.any()
    b1_ref, _ = orc.binarize(th1.astype(np.float64), mode)
    assert np.array_equal(tsat.unpack_bits(solver.get_bits(), N), b1_ref)
    assert solver.get_adam_origin() == 361
    # iteration 361: the fresh optimizer's first update, on the GPU's own gradient
    _, g1 = solver.get_grad(p)
    rep = solver.step(1, params=p)
    assert rep.steps_done == 1
    th2, m2, v2, _ = solver.get_state()
    th_r, m_r, v_r, lr = adam_reference(th1, m1, v1, g1, 361, p, count=1)
    bt, bm, bv = adam_bounds(th1, m1, v1, g1, 361, p, lr, v_r, count=1)
    assert (np.abs(m2 - m_r) <= TOL_ADAM * bm + 1e-30).all()
    assert (np.abs(v2 - v_r) <= TOL_ADAM * bv + 1e-30).all()
    assert (np.abs(th2 - th_r) <= TOL_ADAM * bt + 1e-30).all(), np.abs(th2 - th_r).max()


def test_mixing_off_and_between_restarts(solver):
    """Without the flag iteration 360 is an ordinary update; with it,
    iterations that are not restarts are ordinary updates."""
    cnf = gen.planted_ksat(300, 1230, 3, seed=23)
    solver.load(cnf)
    N = 64
    th, m, v = make_state(300, N, 4100)
    for t, mix in ((360, 0), (359, 1), (0, 1)):
        solver.init_batch(N, init_logits=th)
        solver.set_state(th, m, v, t)
        solver.step(1, params=tsat.default_params(mix=mix))
        _, m1, _, _ = solver.get_state()
        assert m1.any()
        assert solver.get_adam_origin() == 0


def test_mixing_per_instance_in_a_batch(solver):
    """A batch of three instances: each mixes into its own best candidate."""
    cnfs = [gen.planted_ksat(150 + 50 * j, 600 + 200 * j, 3, seed=30 + j) for j in range(3)]
    solver.load_batch(cnfs)
    N = 32
    states = [make_state(c.num_vars, N, 4200 + j) for j, c in enumerate(cnfs)]
    th = np.concatenate([s[0] for s in states])
    m = np.concatenate([s[1] for s in states])
    v = np.concatenate([s[2] for s in states])
    p = tsat.default_params(norm_mode=tsat.MODE_NONE, mix=1)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, 720)
    solver.step(1, params=p)
    th1, m1, v1, _ = solver.get_state()
    assert not m1.any() and not v1.any()
    r0 = 0
    for j, c in enumerate(cnfs):
        ref = orc.step(orc.Cnf.from_gen(c), states[j][0].astype(np.float64), states[j][1].astype(np.float64),
                       states[j][2].astype(np.float64), 720, oparams(p, mix=1))
        assert np.array_equal(th1[r0:r0 + c.num_vars], ref["theta"].astype(np.float32))
        r0 += c.num_vars


def test_adam_origin_checkpoint(solver):
    """Checkpoint/resume across a mixing: state plus the optimizer origin
    reproduce the next iteration bitwise."""
    cnf = gen.planted_ksat(200, 800, 3, seed=24)
    solver.load(cnf)
    N = 64
    th, m, v = make_state(200, N, 4300)
    p = tsat.default_params(mix=1)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, 358)
    solver.step(5, params=p)  # 358, 359, 360 (mixing), 361, 362
    ck = solver.get_state()
    origin = solver.get_adam_origin()
    assert origin == 361 and ck[3] == 363
    solver.step(1, params=p)
    after = solver.get_state()
    solver.set_state(*ck)
    assert solver.get_adam_origin() == 0
    solver.set_adam_origin(origin)
    solver.step(1, params=p)
    again = solver.get_state()
    for a, b in zip(after[:3], again[:3]):
        assert np.array_equal(a, b)
    with pytest.raises(tsat.TsatError):
        solver.set_adam_origin(ck[3] + 5)
