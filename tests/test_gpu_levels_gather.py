"""The clause-plane update for mixed widths (and uniform widths 1 and 4 .. 15)
against the FP64 oracle, one iteration from identical state.

The forward leaves R of every clause in binary (2 planes up to width 3, else
4) and the update counts, per level r and candidate, the records whose clause
has R >= r.  The cases cover every level template of the kernel (widest
clause 3, 4, 8, 12 and 15), rows of one, two and four words, ragged
candidate counts, unit clauses, duplicates, tautologies, variables without
occurrences and variables whose records span many 64-record windows, and a
batch (one dL/dR table per wave).  Expected values come only from the oracle.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

from parity_util import TOL_GRAD, abs_adjoint, grad_bound, make_state, one_step_parity, solver_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    s = solver_or_skip()
    yield s
    s.close()


def width_mix_cnf(widths, V=500, per_width=120, seed=0, heavy=True):
    """Planted clauses of the given widths (distinct variables), plus edge
    clauses when there is more than one width; variable 1 also occurs in 300
    more clauses of each sign so its records span several windows; the last
    5 variables never occur."""
    g = np.random.default_rng(seed)
    z = g.integers(0, 2, size=V)
    Vo = V - 5
    clauses = []
    for k in widths:
        n = 0
        while n < per_width:
            vs = g.choice(Vo, size=k, replace=False)
            sg = g.integers(0, 2, size=k)
            if not (sg == z[vs]).any():
                continue
            clauses.append([int(v + 1) if s else -int(v + 1) for v, s in zip(vs, sg)])
            n += 1
    if heavy:
        for sign in (1, -1):
            for _ in range(300):
                k = int(g.choice(widths))
                others = g.choice(np.arange(2, Vo + 1), size=k - 1, replace=False) if k > 1 else []
                clauses.append([sign] + [int(x) * int(g.choice([-1, 1])) for x in others])
    if len(widths) > 1:  # unit clauses, a duplicate literal, a tautology
        clauses += [[3], [-4], [5, 5, -7], [9, -9, 10]]
    return gen.CNF.from_clauses(V, clauses)


CASES = {
    "w123": [1, 2, 3],
    "uniform4": [4],
    "w2to8": [2, 3, 4, 5, 6, 7, 8],
    "w2to12": list(range(2, 13)),
    "w1to15": list(range(1, 16)),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("N", [64, 100])
def test_levels_gather_one_step(solver, case, N):
    cnf = width_mix_cnf(CASES[case], seed=len(CASES[case]))
    one_step_parity(solver, cnf, N, 4000 + N + len(CASES[case]), 9)


@pytest.mark.parametrize("N", [1, 9, 128, 200, 256])
def test_levels_gather_candidate_counts(solver, N):
    cnf = width_mix_cnf(CASES["w1to15"], seed=15)
    one_step_parity(solver, cnf, N, 4100 + N, 40)


def test_levels_gather_none_mode_and_tau(solver):
    cnf = width_mix_cnf(CASES["w2to12"], seed=3)
    p = tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)
    one_step_parity(solver, cnf, 128, 4200, 3, p=p)


def test_levels_gather_equals_record_gather_up_to_rounding(solver):
    """The same iteration with the clause planes off (records of the other
    literal codes): U and g agree to the gradient tolerance."""
    cnf = width_mix_cnf(CASES["w2to12"], seed=5)
    N = 128
    th, m, v = make_state(cnf.num_vars, N, 4300)
    out = []
    for planes in (1, 0):
        solver.load(cnf)
        solver.set_launch_config(clause_planes=planes, window_gather=1)
        solver.init_batch(N, init_logits=th)
        solver.set_state(th, m, v, 5)
        U, g = solver.get_grad()
        solver.step(1)
        out.append((U, g, solver.get_bits()))
    solver.set_launch_config(clause_planes=1, window_gather=1)
    oc = orc.Cnf.from_gen(cnf)
    b, mu = orc.binarize(th.astype(np.float64))
    _, table, _ = orc.smoothmin(orc.histogram(oc, b), 1.0)
    aU = abs_adjoint(oc, b, table)
    assert (np.abs(out[0][0] - out[1][0]) <= 2 * TOL_GRAD * aU + 1e-30).all()
    g_ref = orc.norm_backward(th.astype(np.float64), orc.adjoint(oc, b, table))
    assert (np.abs(out[0][1] - out[1][1]) <= 2 * TOL_GRAD * grad_bound(aU, th, mu, g_ref) + 1e-30).all()


def test_levels_gather_batch_per_instance(solver):
    """A batch of mixed-width instances: one dL/dR table per wave."""
    cnfs = [width_mix_cnf(CASES["w2to8"], V=300, seed=21), width_mix_cnf(CASES["w1to15"], V=420, seed=22),
            gen.planted_ksat(200, 800, 3, seed=23)]
    N = 64
    parts = [make_state(c.num_vars, N, 4400 + j) for j, c in enumerate(cnfs)]
    th, m, v = (np.concatenate([p[k] for p in parts]) for k in range(3))
    solver.load_batch(cnfs)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, 11)
    U, g = solver.get_grad()
    base = 0
    for j, c in enumerate(cnfs):
        r = slice(base, base + c.num_vars)
        base += c.num_vars
        oc = orc.Cnf.from_gen(c)
        b, mu = orc.binarize(th[r].astype(np.float64))
        _, table, _ = orc.smoothmin(orc.histogram(oc, b), 1.0)
        U_ref = orc.adjoint(oc, b, table)
        aU = abs_adjoint(oc, b, table)
        assert (np.abs(U[r] - U_ref) <= TOL_GRAD * aU + 1e-30).all(), j
        g_ref = orc.norm_backward(th[r].astype(np.float64), U_ref)
        assert (np.abs(g[r] - g_ref) <= TOL_GRAD * grad_bound(aU, th[r], mu, g_ref) + 1e-30).all(), j
