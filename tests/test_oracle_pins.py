"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test ties one oracle function to something fixed independently: values
the paper states for its worked example, brute-force enumeration, closed
forms and invariants of the definitions, a library routine (scipy softmax,
torch.optim.AdamW), or finite differences of a separately written objective.
A plausible slip in the oracle (a dropped term, a wrong sign or index, a
transposed operand) makes at least one of them fail; the ``test_sensitivity_*``
tests show that for representative slips.
"""
import itertools
import json
import os

import numpy as np
import pytest

from paper_2511_07737_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def naive_clause_true_count(clause, assign):
    """Number of true literals of a clause under a dict/array assignment (0/1 per 1-based var)."""
    return sum((assign[abs(x) - 1] == 1) if x > 0 else (assign[abs(x) - 1] == 0) for x in set(clause))


def all_assignments_matrix(n):
    """b[v][i] = bit v of i, for i in 0..2^n-1."""
    i = np.arange(1 << n)
    return ((i[None, :] >> np.arange(n)[:, None]) & 1).astype(np.uint8)


def small_mixed_cnf():
    """Mixed widths, a duplicate literal, a tautology and a unit clause."""
    clauses = [[1, -2, 3], [2, 2, -4], [-1, 5], [4], [3, -3, 6], [-5, -6, 1, 2], [6, -1, -2, 3, -4],
               [-3, 4, 5], [2, -5, -6], [1, 4, -6, 5]]
    return gen.CNF.from_clauses(6, clauses)


# --------------------------------------------------------------------------
# Worked example (Sec. III-A)
# --------------------------------------------------------------------------

def test_worked_example_fragments(orc):
    fx = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    ids = sorted(fx["clauses"], key=int)
    clauses = [fx["clauses"][c]["lits"] for c in ids]
    cnf = orc.Cnf.from_gen(gen.CNF.from_clauses(fx["num_vars"], clauses))
    V = fx["num_vars"]
    aids = sorted(fx["assignments"], key=int)
    # fill the unknown variables every possible way: the stated entries must hold for all fillings
    unknown = {a: [v for v in range(1, V + 1) if str(v) not in fx["assignments"][a]["known"]] for a in aids}
    fills = list(itertools.product(*[list(itertools.product([0, 1], repeat=len(unknown[a]))) for a in aids]))
    assert len(fills) > 1
    for fill in fills:
        b = np.zeros((V, len(aids)), dtype=np.uint8)
        for col, a in enumerate(aids):
            for v, x in fx["assignments"][a]["known"].items():
                b[int(v) - 1, col] = x
            for v, x in zip(unknown[a], fill[col]):
                b[v - 1, col] = x
        R = orc.result_matrix(cnf, b)
        for e in fx["result_entries"]:
            row = ids.index(str(e["clause"]))
            col = aids.index(str(e["assignment"]))
            assert R[row, col] == e["R"], e
    # clause 2 occupies exactly the x3 and x4 columns of P (column 2v for x_v, 2v+1 for not-x_v)
    off, lit = cnf.clauses()
    row2 = lit[off[0]:off[1]]
    P_row = np.zeros(2 * V, dtype=int)
    for x in row2:
        P_row[2 * (abs(x) - 1) + (0 if x > 0 else 1)] = 1
    assert list(np.nonzero(P_row)[0]) == [4, 6]


# --------------------------------------------------------------------------
# R, histogram and the exact check against brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,m,seed,planted", [(8, 34, 1, True), (10, 43, 2, True), (9, 54, 3, False),
                                              (10, 60, 4, False), (7, 50, 5, False)])
def test_check_matches_enumeration(orc, n, m, seed, planted):
    cnf = gen.planted_ksat(n, m, 3, seed) if planted else gen.random_ksat(n, m, 3, seed)
    oc = orc.Cnf.from_gen(cnf)
    b = all_assignments_matrix(n)
    sat, ok = orc.check(oc, b)
    clauses = [list(cnf.clause(c)) for c in range(cnf.num_clauses)]
    for i in range(b.shape[1]):
        a = b[:, i]
        counts = [naive_clause_true_count(cl, a) for cl in clauses]
        assert sat[i] == sum(c > 0 for c in counts)
        assert ok[i] == int(all(c > 0 for c in counts))
    if planted:
        zi = int(sum(int(cnf.planted[v]) << v for v in range(n)))
        assert ok[zi] == 1
    # model count from enumeration equals the number of all-satisfying columns of H
    H = orc.histogram(oc, b)
    assert int((H[:, 0] == 0).sum()) == int(ok.sum())


def test_result_matrix_and_histogram_invariants(orc):
    cnf = small_mixed_cnf()
    oc = orc.Cnf.from_gen(cnf)
    assert oc.K == 5 and oc.L == cnf.num_lits - 1  # the repeated literal 2 is removed
    b = all_assignments_matrix(6)
    R = orc.result_matrix(oc, b)
    clauses = [list(cnf.clause(c)) for c in range(cnf.num_clauses)]
    for i in range(b.shape[1]):
        for c, cl in enumerate(clauses):
            assert R[c, i] == naive_clause_true_count(cl, b[:, i])
    H = orc.histogram(oc, b)
    assert (H.sum(axis=1) == oc.C).all()
    assert (H @ np.arange(oc.K + 1) == R.sum(axis=0)).all()
    # the tautology (3 or not 3 or 6) always has a true literal
    assert (R[4] >= 1).all()
    # the exact check is "column minimum of R nonzero"
    sat, ok = orc.check(oc, b)
    assert (ok == (R.min(axis=0) > 0)).all()
    assert (sat == (R > 0).sum(axis=0)).all()


def test_planted_assignment_satisfies_every_clause(orc):
    for seed in range(3):
        cnf = gen.planted_ksat(300, 1300, 3, seed)
        oc = orc.Cnf.from_gen(cnf)
        sat, ok = orc.check(oc, cnf.planted[:, None])
        assert ok[0] == 1 and sat[0] == oc.C
    s = gen.structured(2000, 9000, seed=5)
    oc = orc.Cnf.from_gen(s)
    sat, ok = orc.check(oc, s.planted[:, None])
    assert ok[0] == 1


def test_empty_clause_and_empty_cnf(orc):
    # an empty clause can never be satisfied
    oc = orc.Cnf(3, np.array([1, 2, 0, 0, -3, 0], dtype=np.int32))
    assert oc.C == 3
    b = all_assignments_matrix(3)
    sat, ok = orc.check(oc, b)
    assert ok.sum() == 0
    # no clauses: every candidate satisfies the (empty) conjunction; S is 0
    oc0 = orc.Cnf(3, np.zeros(0, dtype=np.int32))
    sat, ok = orc.check(oc0, b)
    assert ok.all() and (sat == 0).all()
    S, table, loss = orc.smoothmin(orc.histogram(oc0, b))
    assert (S == 0).all() and loss == 0 and (table == 0).all()


# --------------------------------------------------------------------------
# SmoothMin (Eq. 4) and the loss (Eq. 3)
# --------------------------------------------------------------------------

def random_hist(seed, N=7, K=4):
    g = np.random.default_rng(seed)
    H = g.integers(0, 40, size=(N, K + 1)).astype(np.int64)
    H[0, :2] = 0  # a column whose minimum is 2
    return H


def expand(H_row):
    return np.repeat(np.arange(H_row.size), H_row).astype(np.float64)


def test_smoothmin_equals_softmax_weighted_mean(orc):
    from scipy.special import softmax

    for tau in (0.0, 0.5, 1.0, 2.0, 7.0):
        H = random_hist(1)
        S, _, loss = orc.smoothmin(H, tau)
        for i in range(H.shape[0]):
            R = expand(H[i])
            assert S[i] == pytest.approx(float(R @ softmax(-tau * R)), rel=1e-13, abs=1e-13)
        assert loss == pytest.approx(-S.sum(), rel=1e-14)


def test_smoothmin_limits_and_bounds(orc):
    H = random_hist(2)
    S0, _, _ = orc.smoothmin(H, 0.0)
    means = [expand(h).mean() for h in H]
    assert np.allclose(S0, means, rtol=1e-14)  # tau = 0: arithmetic mean
    Sinf, _, _ = orc.smoothmin(H, 60.0)
    mins = [expand(h).min() for h in H]
    assert np.allclose(Sinf, mins, atol=1e-15)  # tau -> infinity: minimum
    for tau in (0.3, 1.0, 3.0):
        S, _, _ = orc.smoothmin(H, tau)
        assert all(mn - 1e-12 <= s <= me + 1e-12 for s, mn, me in zip(S, mins, means))
    Hc = np.zeros((3, 5), dtype=np.int64)
    Hc[:, 2] = 11  # constant column R = 2
    Sc, _, _ = orc.smoothmin(Hc, 1.7)
    assert np.allclose(Sc, 2.0, rtol=0, atol=1e-15)


def test_smoothmin_shift_equivariance_sum_rule(orc):
    """S(R + c) = S(R) + c, hence sum_c dS_i/dR_ci = 1: the dL/dR table sums
    to the upstream gradient (-1 for the loss) over every clause."""
    for tau in (0.5, 1.0, 2.0):
        H = random_hist(3)
        _, table, _ = orc.smoothmin(H, tau)
        assert np.allclose((H * table).sum(axis=1), -1.0, atol=1e-13)
        dS = np.linspace(-2, 3, H.shape[0])
        _, table2, _ = orc.smoothmin(H, tau, dS)
        assert np.allclose((H * table2).sum(axis=1), dS, atol=1e-13)
        # shifting every R of a column by one leaves the table shape, moves S by one
        Hs = np.zeros((H.shape[0], H.shape[1] + 1), dtype=np.int64)
        Hs[:, 1:] = H
        S, _, _ = orc.smoothmin(H, tau)
        S1, _, _ = orc.smoothmin(Hs, tau)
        assert np.allclose(S1, S + 1, rtol=1e-14)


def test_histogram_smoothmin_matches_direct_eq4(orc):
    """The histogram/shifted evaluation equals Eq. 4 summed clause by clause."""
    cnf = small_mixed_cnf()
    oc = orc.Cnf.from_gen(cnf)
    b = all_assignments_matrix(6)[:, ::5]
    H = orc.histogram(oc, b)
    for tau in (0.5, 1.0, 3.0):
        S, _, _ = orc.smoothmin(H, tau)
        for i in range(b.shape[1]):
            assert orc.relaxed_S(oc, b.astype(np.float64), i, tau) == pytest.approx(S[i], rel=1e-13)


# --------------------------------------------------------------------------
# Gradient: STE adjoint and the Eq. 5 backward
# --------------------------------------------------------------------------

def fd_relaxed(orc, oc, x, tau, h=1e-4):
    """Central differences of the relaxed loss -sum_i S~_i with respect to every x_vi."""
    V, N = x.shape
    G = np.zeros_like(x)
    for v in range(V):
        for i in range(N):
            xp = x.copy(); xp[v, i] += h
            xm = x.copy(); xm[v, i] -= h
            G[v, i] = -(orc.relaxed_S(oc, xp, i, tau) - orc.relaxed_S(oc, xm, i, tau)) / (2 * h)
    return G


@pytest.mark.parametrize("tau", [0.5, 1.0, 2.0])
def test_adjoint_is_exact_gradient_of_relaxed_loss(orc, tau):
    """At a binary point the straight-through gradient dL/dtheta_norm equals the
    exact gradient of L~(x) = -sum_i SmoothMin(P [x; 1-x])_i (Eqs. 1, 3, 4)."""
    for cnf in (small_mixed_cnf(), gen.planted_ksat(12, 50, 3, 7)):
        oc = orc.Cnf.from_gen(cnf)
        theta = gen.normal_logits(cnf.num_vars, 5, 11).astype(np.float64)
        b, _ = orc.binarize(theta, orc.MODE_NONE)
        H = orc.histogram(oc, b)
        _, table, _ = orc.smoothmin(H, tau)
        U = orc.adjoint(oc, b, table)
        G = fd_relaxed(orc, oc, b.astype(np.float64), tau)
        assert np.allclose(U, G, rtol=1e-6, atol=1e-9), np.abs(U - G).max()


def test_relaxed_fd_matches_naive_central_difference(orc):
    """The cancellation-free central difference equals the plain one where
    the plain one is accurate (small instances), and both converge onto the
    adjoint U as h -> 0."""
    cnf = small_mixed_cnf()
    oc = orc.Cnf.from_gen(cnf)
    b, _ = orc.binarize(gen.normal_logits(6, 5, 3).astype(np.float64), orc.MODE_NONE)
    x = b.astype(np.float64)
    _, table, _ = orc.smoothmin(orc.histogram(oc, b), 1.3)
    U = orc.adjoint(oc, b, table)
    for v in range(6):
        for i in range(5):
            for h in (1e-2, 1e-3):
                xp = x.copy(); xp[v, i] += h
                xm = x.copy(); xm[v, i] -= h
                naive = (orc.relaxed_S(oc, xp, i, 1.3) - orc.relaxed_S(oc, xm, i, 1.3)) / (2 * h)
                assert orc.relaxed_fd(oc, x, v, i, h, 1.3) == pytest.approx(naive, rel=1e-9, abs=1e-12)
            # -dS~/dx = U (Eq. 3 sign); O(h^2) convergence
            e3 = abs(-orc.relaxed_fd(oc, x, v, i, 1e-3, 1.3) - U[v, i])
            e4 = abs(-orc.relaxed_fd(oc, x, v, i, 1e-4, 1.3) - U[v, i])
            assert e4 <= max(e3 / 50, 1e-13)


def test_norm_backward_matches_fd(orc):
    """g = d/dtheta <U, theta / mean_row(theta)> with U held fixed (Eq. 5)."""
    g0 = np.random.default_rng(4)
    V, N = 6, 9
    theta = g0.normal(size=(V, N)) + 0.3
    U = g0.normal(size=(V, N))
    g = orc.norm_backward(theta, U, orc.MODE_MEAN)

    def phi(th):
        return float((U * (th / th.mean(axis=1, keepdims=True))).sum())

    h = 1e-6
    for v in range(V):
        for i in range(N):
            tp = theta.copy(); tp[v, i] += h
            tm = theta.copy(); tm[v, i] -= h
            fd = (phi(tp) - phi(tm)) / (2 * h)
            assert g[v, i] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    # degree-0 homogeneity of theta / mean(theta): sum_i theta_vi g_vi = 0
    assert np.allclose((theta * g).sum(axis=1), 0.0, atol=1e-12)
    # none mode: the identity
    assert np.array_equal(orc.norm_backward(theta, U, orc.MODE_NONE), U)


def test_norm_backward_clamped_row(orc):
    """A row with zero mean uses mu = +1e-12 and no d(mu) term (clamp is flat there)."""
    theta = np.array([[1.0, -1.0, 2.0, -2.0], [0.5, 0.1, 0.2, 0.3]])
    U = np.array([[1.0, 2.0, 3.0, 4.0], [1.0, 1.0, 1.0, 1.0]])
    g = orc.norm_backward(theta, U)
    assert np.allclose(g[0], U[0] / 1e-12, rtol=1e-15)
    b, mu = orc.binarize(theta)
    assert mu[0] == 1e-12 and list(b[0]) == [1, 0, 1, 0]


# --------------------------------------------------------------------------
# Binarization (Eq. 2 with Eq. 5)
# --------------------------------------------------------------------------

def test_binarize_definition_and_balance(orc):
    theta = np.array([[0.0, 1.0, -1.0, 2.0], [-3.0, 1.0, 0.0, 1.0], [0.0, 0.0, 0.0, 0.0]])
    b, mu = orc.binarize(theta, orc.MODE_NONE)
    assert b.tolist() == [[0, 1, 0, 1], [0, 1, 0, 1], [0, 0, 0, 0]]  # B(0) = 0
    b, mu = orc.binarize(theta, orc.MODE_MEAN)
    # row 1 has negative mean: the normalized entries are positive where theta < 0
    assert b.tolist() == [[0, 1, 0, 1], [1, 0, 0, 0], [0, 0, 0, 0]]
    assert mu[0] == pytest.approx(0.5) and mu[1] == pytest.approx(-0.25)
    # N(0,1) init gives balanced bits in none mode (Sec. IV-A)
    th = gen.normal_logits(4000, 64, 5).astype(np.float64)
    b, _ = orc.binarize(th, orc.MODE_NONE)
    assert abs(b.mean() - 0.5) < 5 * 0.5 / np.sqrt(b.size)
    # mean mode: the normalized row has mean 1, so every variable is True somewhere
    b, mu = orc.binarize(th, orc.MODE_MEAN)
    assert (b.max(axis=1) == 1).all()
    assert np.array_equal(b, ((th > 0) == (mu[:, None] > 0)) & (th != 0))


# --------------------------------------------------------------------------
# Optimizer and schedule (Sec. IV-A)
# --------------------------------------------------------------------------

def test_lr_schedule_values(orc):
    expect = {0: 0.1, 29: 0.1, 30: 0.01, 59: 0.01, 60: 1e-3, 329: 1e-11, 330: 1e-12, 359: 1e-12,
              360: 0.1, 389: 0.1, 390: 0.01, 720: 0.1}
    for t, want in expect.items():
        assert orc.lr(t) == pytest.approx(want, rel=1e-12), t
    assert min(orc.lr(t) for t in range(2000)) >= 1e-15


def test_adamw_matches_torch(orc):
    torch = pytest.importorskip("torch")
    g0 = np.random.default_rng(8)
    n = 200
    theta = g0.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    p = torch.tensor(theta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([p], lr=0.1, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-2)
    for t in range(70):
        grad = g0.normal(size=n) * (10.0 ** g0.integers(-6, 2))
        lr = orc.lr(t)
        for group in opt.param_groups:
            group["lr"] = lr
        p.grad = torch.tensor(grad, dtype=torch.float64)
        opt.step()
        orc.adamw(theta, m, v, grad, lr, t + 1)
        assert np.allclose(theta, p.detach().numpy(), rtol=1e-13, atol=1e-15), t


def test_adamw_first_step_closed_form(orc):
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -1e-3, 1e-9])
    m = np.zeros(3); v = np.zeros(3)
    expected = theta * (1 - 0.1 * 1e-2) - 0.1 * g / (np.abs(g) + 1e-8)
    orc.adamw(theta, m, v, g, 0.1, 1)
    assert np.allclose(theta, expected, rtol=1e-12)


def test_step_is_the_composition(orc):
    cnf = gen.planted_ksat(30, 120, 3, 9)
    oc = orc.Cnf.from_gen(cnf)
    th = gen.normal_logits(30, 8, 21).astype(np.float64)
    m = np.abs(gen.normal_logits(30, 8, 22).astype(np.float64)) * 0.01
    v = np.abs(gen.normal_logits(30, 8, 23).astype(np.float64)) * 0.01
    t = 37
    out = orc.step(oc, th, m, v, t)
    b, _ = orc.binarize(th)
    H = orc.histogram(oc, b)
    S, table, loss = orc.smoothmin(H, 1.0)
    U = orc.adjoint(oc, b, table)
    g = orc.norm_backward(th, U)
    th2, m2, v2 = th.copy(), m.copy(), v.copy()
    orc.adamw(th2, m2, v2, g, orc.lr(t), t + 1)
    assert np.array_equal(out["bits"], b) and np.array_equal(out["H"], H)
    assert out["loss"] == loss and np.array_equal(out["g"], g)
    assert np.array_equal(out["theta"], th2) and np.array_equal(out["v"], v2)


# --------------------------------------------------------------------------
# Handoff (Sec. IV-B)
# --------------------------------------------------------------------------

def test_extract_partial_against_lexsort(orc):
    cnf = gen.planted_ksat(60, 200, 3, 12)
    # variable 60 never occurs: drop its clauses
    keep = [c for c in range(cnf.num_clauses) if 60 not in np.abs(cnf.clause(c))]
    cnf = gen.CNF.from_clauses(60, [cnf.clause(c) for c in keep])
    oc = orc.Cnf.from_gen(cnf)
    g0 = np.random.default_rng(3)
    N = 10
    g = np.round(g0.normal(size=(60, N)), 1)  # many ties
    b = g0.integers(0, 2, size=(60, N)).astype(np.uint8)
    sat = g0.integers(190, 200, size=N).astype(np.int64)
    k = orc.default_k(60)
    ids, lits, so = orc.extract_partial(oc, g, b, sat, 6, k)
    order = np.lexsort((np.arange(N), -sat))
    assert list(ids) == list(order[:6])
    occurs = np.zeros(60, bool)
    occurs[np.abs(cnf.lits) - 1] = True
    for a, i in enumerate(ids):
        vs = np.nonzero(occurs)[0]
        sel = vs[np.lexsort((vs, np.abs(g[vs, i])))][:k]
        want = np.where(b[sel, i] == 1, sel + 1, -(sel + 1))
        assert list(lits[a]) == list(want)
        assert so[a] == sat[i]
    assert k == 20 and orc.default_k(1_000_000) == 100 and orc.default_k(200_001) == 21


# --------------------------------------------------------------------------
# Sensitivity: plausible slips, made on the CPU, fail the pins above
# --------------------------------------------------------------------------

def test_sensitivity_dropped_term_in_table_fails_fd(orc):
    cnf = gen.planted_ksat(12, 50, 3, 7)
    oc = orc.Cnf.from_gen(cnf)
    b, _ = orc.binarize(gen.normal_logits(12, 4, 11).astype(np.float64), orc.MODE_NONE)
    H = orc.histogram(oc, b)
    S, table, _ = orc.smoothmin(H, 1.0)
    G = fd_relaxed(orc, oc, b.astype(np.float64), 1.0)
    r = np.arange(H.shape[1])[None, :]
    w = np.exp(-(r - (H > 0).argmax(axis=1)[:, None]))
    D = (H * w).sum(axis=1, keepdims=True)
    bad_tables = [
        -(w / D) * (1 - r),  # tau*S term dropped
        (w / D) * (1 - (r - S[:, None])),  # sign of the loss flipped
        -(w / D),  # derivative of the numerator only
    ]
    for bad in bad_tables:
        U_bad = orc.adjoint(oc, b, bad)
        assert not np.allclose(U_bad, G, rtol=1e-6, atol=1e-9)
    # transposed candidates (wrong column of the table) also fail
    U_t = orc.adjoint(oc, b, table[::-1].copy())
    assert not np.allclose(U_t, G, rtol=1e-6, atol=1e-9)


def test_sensitivity_norm_backward_without_mean_term_fails_invariant(orc):
    g0 = np.random.default_rng(5)
    theta = g0.normal(size=(4, 6)) + 0.5
    U = g0.normal(size=(4, 6))
    bad = U / theta.mean(axis=1, keepdims=True)  # mean treated as a constant
    assert not np.allclose((theta * bad).sum(axis=1), 0.0, atol=1e-8)
