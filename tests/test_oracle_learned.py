"""Pins of the oracle's learned-proposal parts: random streams, proposal
initialisation, per-variable features and the FP64 network.

Each check ties a function to something outside itself: published known-answer
vectors of Philox4x32-10, distribution tests, the defining property of the
initialisation (Eq. 5 then Eq. 2 give back the drawn bits), hand-computed
features, a dense-matrix restatement of the aggregation, symmetries, torch's
bfloat16 conversion, torch float64 autograd and torch.optim.Adam.
"""
import numpy as np
import pytest

import oracle as orc
from oracle import mlp
from paper_2511_07737_amd import gen


# --------------------------------------------------------------------------
# Philox4x32-10 and the N(0,1) / Bernoulli streams
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ctr,key,expect", [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
])
def test_philox_known_answers(ctr, key, expect):
    """Known-answer vectors published with the Random123 library (Salmon et al., SC'11)."""
    assert list(orc.philox4x32_10(ctr, key)) == expect


def test_init_normal_distribution():
    from scipy import stats

    th = orc.init_normal(400, 256, 1234).ravel()
    assert th.dtype == np.float32
    assert abs(th.mean()) < 0.01 and abs(th.std() - 1) < 0.01
    assert stats.kstest(th.astype(np.float64), "norm").pvalue > 1e-3
    # seeds give different, reproducible streams
    assert np.array_equal(th, orc.init_normal(400, 256, 1234).ravel())
    assert not np.array_equal(th[:1000], orc.init_normal(400, 256, 1235).ravel()[:1000])


def test_proposal_bits_follow_p_and_magnitudes_match_random_init():
    from scipy import stats

    V, N, seed = 300, 128, 77
    p = np.linspace(0, 1, V).astype(np.float32)
    z = orc.init_normal(V, N, seed)
    th = orc.init_proposal(p, N, seed, orc.MODE_NONE)
    assert np.array_equal(np.abs(th), np.abs(z))
    b = (th > 0).astype(np.uint8)
    assert b[0].sum() == 0 and b[-1].sum() == N  # p = 0 and p = 1
    # row frequencies are binomial(N, p_v): a chi-square over all rows
    k = b.sum(axis=1).astype(np.float64)
    mid = (p > 0) & (p < 1)
    pm = p[mid].astype(np.float64)
    chi2 = (((k[mid] - N * pm) ** 2) / (N * pm * (1 - pm))).sum()
    assert stats.chi2.sf(chi2, mid.sum()) > 1e-4


@pytest.mark.parametrize("mode", [0, 1])
def test_proposal_init_is_reproduced_by_binarization(mode):
    """The defining property: Eq. 5 (mode) followed by Eq. 2 returns the drawn bits."""
    V, N, seed = 500, 64, 9
    g = np.random.default_rng(0)
    p = g.uniform(0, 1, V).astype(np.float32)
    p[:20] = 0.0
    p[20:40] = 1.0
    p[40:60] = 1e-3
    th = orc.init_proposal(p, N, seed, mode)
    b_drawn = (th > 0).astype(np.uint8)
    b, mu = orc.binarize(th.astype(np.float64), mode)
    assert np.array_equal(b, b_drawn)
    if mode == 1:
        assert (mu > 0).all()
        assert (b.sum(axis=1) >= 1).all()
        # all-false rows are repaired at candidate v mod N and nowhere else
        for v in range(20):
            assert list(np.nonzero(b[v])[0]) == [v % N]
    else:
        assert b[:20].sum() == 0


def test_proposal_mean_mode_scaling_only_touches_negatives():
    V, N, seed = 200, 32, 5
    p = np.full(V, 0.2, dtype=np.float32)
    z = np.abs(orc.init_normal(V, N, seed))
    th = orc.init_proposal(p, N, seed, orc.MODE_MEAN)
    pos = th > 0
    assert np.array_equal(th[pos], z[pos])
    ratio = -th[~pos] / z[~pos]
    assert (ratio > 0).all() and (ratio <= 1).all()
    # per row the negative entries share one factor rho <= 1, and mu > 0
    for v in range(V):
        r = -th[v][~pos[v]] / z[v][~pos[v]]
        if r.size:
            assert np.ptp(r) <= 2e-7 * r.max()
        assert th[v].astype(np.float64).mean() > 0


# --------------------------------------------------------------------------
# Per-variable features
# --------------------------------------------------------------------------

def test_features_hand_example():
    # clauses: (1 2) (-1 3) (1 -2 3) and the tautology (2 -2 3), ignored
    clauses = [[1, 2], [-1, 3], [1, -2, 3], [2, -2, 3]]
    oc = orc.Cnf.from_gen(gen.CNF.from_clauses(3, clauses))
    X = orc.features(oc)
    # var 1: pos 2, neg 1; var 2: pos 1, neg 1; var 3: pos 2, neg 0
    assert X[0, 0] == pytest.approx(np.log(3)) and X[0, 1] == pytest.approx(np.log(2))
    assert X[0, 2] == pytest.approx(1 / 3) and X[1, 2] == 0 and X[2, 2] == 1
    # mean widths / 4: var1 (2+2+3)/3, var2 (2+3)/2, var3 (2+3)/2
    assert X[0, 3] == pytest.approx(7 / 12) and X[1, 3] == pytest.approx(5 / 8) and X[2, 3] == pytest.approx(5 / 8)
    # round 1, channel 3 (h0 = 1): sum of sign products over co-literals / Z
    # var1: (1 2): +1; (-1 3): -1; (1 -2 3): -1 + 1 -> total 0 over Z = 4
    # var2: (1 2): +1; (1 -2 3): -1 -1 -> total -1 over Z = 3
    # var3: (-1 3): -1; (1 -2 3): +1 -1 -> total -1 over Z = 3
    assert X[0, 7] == pytest.approx(0.0) and X[1, 7] == pytest.approx(-1 / 3) and X[2, 7] == pytest.approx(-1 / 3)
    # round 1, channel 0 (h0 = polarity bias [1/3, 0, 1]):
    # var1: (+1)(0) + (-1)(1) + [(-1)(0) + (+1)(1)] = 0 -> 0/4
    # var2: (+1)(1/3) + [(-1)(1/3) + (-1)(1)] = -1 -> -1/3
    # var3: (-1)(1/3) + [(+1)(1/3) + (-1)(0)] = 0 -> 0
    assert X[0, 4] == pytest.approx(0.0) and X[1, 4] == pytest.approx(-1 / 3) and X[2, 4] == pytest.approx(0.0)


def dense_features(cnf):
    """The same features through a dense signed co-occurrence matrix M[v][u]
    and h_r = diag(1/max(1,Z)) M h_{r-1}: a second statement of the definition."""
    V = cnf.num_vars
    M = np.zeros((V, V))
    Z = np.zeros(V)
    pos = np.zeros(V)
    neg = np.zeros(V)
    wsum = np.zeros(V)
    for c in range(cnf.num_clauses):
        cl = sorted(set(int(x) for x in cnf.clause(c)))
        if any(-x in cl for x in cl):
            continue
        for x in cl:
            v = abs(x) - 1
            (pos if x > 0 else neg)[v] += 1
            wsum[v] += len(cl)
            for y in cl:
                if abs(y) != abs(x):
                    M[v, abs(y) - 1] += np.sign(x) * np.sign(y)
                    Z[v] += 1
    Z = np.maximum(1, Z)
    deg = pos + neg
    h = np.stack([(pos - neg) / np.maximum(1, deg), (pos - neg) / np.sqrt(np.maximum(1, deg)),
                  np.log1p(pos) - np.log1p(neg), np.ones(V)], axis=1)
    cols = [np.log1p(pos), np.log1p(neg), (pos - neg) / np.maximum(1, deg),
            np.where(deg > 0, wsum / np.maximum(deg, 1) / 4, 0.0)]
    out = [np.stack(cols, axis=1)]
    for _ in range(3):
        h = (M @ h) / Z[:, None]
        out.append(h)
    return np.concatenate(out, axis=1)


@pytest.mark.parametrize("maker", [
    lambda: gen.planted_ksat(60, 250, 3, seed=4),
    lambda: gen.random_ksat(40, 170, 3, seed=5),
    lambda: gen.structured(300, 1200, seed=6, communities=8),
])
def test_features_match_dense_restatement(maker):
    cnf = maker()
    X = orc.features(orc.Cnf.from_gen(cnf))
    np.testing.assert_allclose(X, dense_features(cnf), rtol=1e-12, atol=1e-12)


def test_features_symmetries():
    cnf = gen.structured(400, 1700, seed=8, communities=8)
    X = orc.features(orc.Cnf.from_gen(cnf))
    # global polarity flip: pos/neg swap, signed channels flip, the constant channel does not
    flip = gen.CNF(cnf.num_vars, cnf.offsets, -cnf.lits, None, {})
    Xf = orc.features(orc.Cnf.from_gen(flip))
    np.testing.assert_allclose(Xf[:, 0], X[:, 1], rtol=1e-13)
    np.testing.assert_allclose(Xf[:, 3], X[:, 3], rtol=1e-13)
    for r in range(4):
        base = 4 * r
        chans = (2,) if r == 0 else (base, base + 1, base + 2)
        for ch in chans:
            np.testing.assert_allclose(Xf[:, ch], -X[:, ch], rtol=1e-12, atol=1e-14)
        if r > 0:
            np.testing.assert_allclose(Xf[:, base + 3], X[:, base + 3], rtol=1e-12, atol=1e-14)
    # variable relabelling permutes the rows
    perm = np.random.default_rng(1).permutation(cnf.num_vars)
    lits = np.sign(cnf.lits) * (perm[np.abs(cnf.lits) - 1] + 1)
    Xp = orc.features(orc.Cnf.from_gen(gen.CNF(cnf.num_vars, cnf.offsets, lits.astype(np.int32), None, {})))
    np.testing.assert_allclose(Xp[perm], X, rtol=1e-12, atol=1e-14)
    # adding tautologies changes nothing; a disjoint union is the stack of its parts
    extra = [[1, -1, 5], [7, -7]]
    c2 = gen.CNF.from_clauses(cnf.num_vars, [list(cnf.clause(c)) for c in range(cnf.num_clauses)] + extra)
    np.testing.assert_array_equal(orc.features(orc.Cnf.from_gen(c2)), X)
    other = gen.planted_ksat(50, 200, 3, seed=2)
    shifted = [[int(np.sign(x)) * (abs(int(x)) + cnf.num_vars) for x in other.clause(c)] for c in range(other.num_clauses)]
    u = gen.CNF.from_clauses(cnf.num_vars + 50, [list(cnf.clause(c)) for c in range(cnf.num_clauses)] + shifted)
    Xu = orc.features(orc.Cnf.from_gen(u))
    np.testing.assert_allclose(Xu[:cnf.num_vars], X, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Xu[cnf.num_vars:], orc.features(orc.Cnf.from_gen(other)), rtol=1e-13, atol=1e-15)


def test_features_of_isolated_variables_are_zero():
    oc = orc.Cnf.from_gen(gen.CNF.from_clauses(5, [[1, 2], [-2, 3]]))
    X = orc.features(oc)
    assert (X[3:] == 0).all()


# --------------------------------------------------------------------------
# The network
# --------------------------------------------------------------------------

def test_bf16_rounding_matches_torch():
    import torch

    g = np.random.default_rng(3)
    x = np.concatenate([g.normal(0, 1, 20000), g.normal(0, 1e-3, 2000), g.normal(0, 50, 2000)]).astype(np.float32)
    # exact ties between two bfloat16 neighbours, both parities
    base = np.float32(1.5) * (2.0 ** np.arange(-6, 7)).astype(np.float32)
    ties = (base.view(np.uint32) + np.uint32(0x8000)).view(np.float32)
    ties2 = (base.view(np.uint32) + np.uint32(0x18000)).view(np.float32)
    x = np.concatenate([x, ties, ties2, -ties, [0.0, -0.0, 1.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x.astype(np.float64)), ref)


def torch_loss(p, X, y, w):
    """The same network and loss written with torch float64 autograd; the
    rounded weights are treated as the leaves (the straight-through reading)."""
    import torch

    T = {k: torch.tensor(mlp.bf16(p[k]) if k in ("W1", "W2", "w3") else p[k], dtype=torch.float64,
                         requires_grad=True) for k in mlp.ORDER}
    xq = torch.tensor(mlp.bf16(X), dtype=torch.float64)
    a1 = xq @ T["W1"] + T["b1"]
    h1 = torch.relu(a1)
    h1q = h1 + (torch.tensor(mlp.bf16(h1.detach().numpy())) - h1).detach()  # rounding with identity gradient
    a2 = h1q @ T["W2"] + T["b2"]
    out = torch.relu(a2) @ T["w3"] + T["b3"]
    lw = torch.nn.functional.binary_cross_entropy_with_logits(out, torch.tensor(y, dtype=torch.float64),
                                                              weight=torch.tensor(w), reduction="sum") / len(y)
    lw.backward()
    return float(lw), {k: T[k].grad.numpy() for k in mlp.ORDER}


def test_network_gradient_matches_torch_autograd():
    g = np.random.default_rng(4)
    p = mlp.init_params(11)
    p["b1"] = g.normal(0, 0.1, 128)
    p["b2"] = g.normal(0, 0.1, 128)
    p["b3"] = np.array([0.3])
    X = g.normal(0, 1, (300, 16))
    y = (g.random(300) < 0.4).astype(np.float64)
    w = g.uniform(0.5, 2, 300)
    loss, grad, f = mlp.loss_and_grad(p, X, y, w)
    tl, tg = torch_loss(p, X, y, w)
    assert loss == pytest.approx(tl, rel=1e-13)
    for k in mlp.ORDER:
        np.testing.assert_allclose(grad[k], tg[k], rtol=1e-11, atol=1e-15)
    # relu masks are taken on h1q: the derivative is 0 where the rounded activation is 0
    assert ((f["h1q"] > 0) == (f["a1"] > 0)).all()


def test_network_gradient_matches_finite_differences_without_rounding():
    g = np.random.default_rng(5)
    p = mlp.init_params(12)
    p["b2"] = g.normal(0, 0.2, 128)
    X = g.normal(0, 1, (64, 16))
    y = (g.random(64) < 0.5).astype(np.float64)
    _, grad, _ = mlp.loss_and_grad(p, X, y, quantize=False)
    flat = mlp.flatten(p)
    gflat = mlp.flatten(grad)
    idx = g.choice(flat.size, 60, replace=False)
    h = 1e-6
    for j in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[j] += h
        fm[j] -= h
        lp = mlp.loss_and_grad(mlp.unflatten(fp), X, y, quantize=False)[0]
        lm = mlp.loss_and_grad(mlp.unflatten(fm), X, y, quantize=False)[0]
        assert (lp - lm) / (2 * h) == pytest.approx(gflat[j], rel=1e-6, abs=1e-10)


def test_network_adam_matches_torch():
    import torch

    g = np.random.default_rng(6)
    p = mlp.init_params(13)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    T = [torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in mlp.ORDER]
    opt = torch.optim.Adam(T, lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        grads = {k: g.normal(0, 1, mlp.SHAPES[k]) for k in mlp.ORDER}
        mlp.adam(p, grads, m, v, t, 3e-3)
        for tt, k in zip(T, mlp.ORDER):
            tt.grad = torch.tensor(grads[k])
        opt.step()
    for tt, k in zip(T, mlp.ORDER):
        np.testing.assert_allclose(p[k], tt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_fragile_rows_flags_ties_and_relu_edges():
    p = mlp.init_params(14)
    X = np.random.default_rng(7).normal(0, 1, (200, 16))
    X = mlp.bf16(X)
    # force an exact zero pre-activation in row 0, unit 0: b1[0] = -(xq @ W1q)[0, 0]
    f = mlp.forward(p, X)
    p["b1"] = p["b1"].copy()
    p["b1"][0] = -(f["xq"] @ f["W1q"])[0, 0]
    flags = mlp.fragile_rows(p, X)
    assert flags[0]
    assert flags.mean() < 0.5
