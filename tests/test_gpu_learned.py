"""GPU parity of the learned proposal against the oracle: features, the
random streams and proposal start, the network's forward pass, gradient and
Adam step.

Tolerances follow from the arithmetic of the GPU path:
  * features: FP32 sums of O(degree) terms per round; 2e-5 relative to the
    magnitude of the value (plus 2e-5 absolute for values near zero);
  * drawn bits: integer comparisons of the same Philox words, exact; theta:
    one FP32 rounding of an FP64 expression, so within one ulp;
  * network forward: BF16 products are exact in FP32; the sums carry at most
    (terms) x 2^-24 of their absolute-value sums, so logits are held to
    2e-5 of the absolute-value scale of the output, on rows whose relu or
    rounding decisions are not within FP32 reach of a boundary (the oracle
    flags those and they are left out);
  * gradient: sums over the batch in FP32, held to 1e-5 of the absolute-value
    sum of the same products (the gradient tolerance of the method's FP32 path).
"""
import numpy as np
import pytest

import oracle as orc
from oracle import mlp
from paper_2511_07737_amd import gen, tsat

from parity_util import solver_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T

    if not T.cuda.is_available():
        pytest.skip("no GPU visible")
    return T


@pytest.fixture
def solver():
    s = solver_or_skip()
    yield s
    s.close()


def mixed_cnf():
    """Mixed widths, tautologies, an empty clause, isolated variables."""
    g = np.random.default_rng(3)
    clauses = []
    for _ in range(900):
        k = int(g.integers(1, 7))
        vs = g.choice(300, size=k, replace=False) + 1
        clauses.append([int(v) if g.random() < 0.5 else -int(v) for v in vs])
    clauses += [[5, -5, 7], [9, -9], [], [11, 12, -11, 13]]
    return gen.CNF.from_clauses(320, clauses)


def check_features(X, ref):
    assert X.shape == ref.shape
    err = np.abs(X.astype(np.float64) - ref)
    lim = 2e-5 * np.abs(ref) + 2e-5
    bad = np.argwhere(err > lim)
    assert bad.size == 0, (bad[:5], X[tuple(bad[0])], ref[tuple(bad[0])])


@pytest.mark.parametrize("maker", [
    lambda: gen.planted_ksat(2000, 8200, 3, seed=11),
    lambda: gen.structured(5000, 22000, seed=12),
    mixed_cnf,
])
def test_features_vs_oracle(solver, maker):
    cnf = maker()
    solver.load(cnf)
    X = solver.get_features()
    check_features(X, orc.features(orc.Cnf.from_gen(cnf)))


def test_features_of_a_batch_are_those_of_its_instances(solver):
    cnfs = [gen.planted_ksat(500, 2050, 3, seed=21), mixed_cnf(), gen.planted_ksat(64, 250, 3, seed=22)]
    solver.load_batch(cnfs)
    X = solver.get_features()
    o = 0
    for c in cnfs:
        check_features(X[o:o + c.num_vars], orc.features(orc.Cnf.from_gen(c)))
        o += c.num_vars
    assert o == X.shape[0]


def test_features_dev_matches_host_call(solver, torch):
    cnf = gen.structured(3000, 13000, seed=13)
    solver.load(cnf)
    X = solver.get_features()
    T = torch.empty((cnf.num_vars, 16), dtype=torch.float32, device="cuda")
    solver.features_dev(T.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert np.array_equal(T.cpu().numpy(), X)


# --------------------------------------------------------------------------
# random streams and the proposal start
# --------------------------------------------------------------------------

def ulp_close(a, b, ulps=1):
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    return np.abs(a.astype(np.float64) - b) <= ulps * np.spacing(np.maximum(np.abs(a), np.abs(b)))


def test_random_init_matches_oracle_stream(solver):
    """Both sides draw the same Philox words and form Box-Muller in FP64,
    rounded to FP32 once; their FP64 log/cos may differ in the last FP64
    bit, which changes the FP32 value only for a draw within that distance
    of an FP32 rounding boundary (about 2^-28 of the draws): the logits agree
    within one FP32 ulp, nearly all of them exactly, and the binarized start
    (Eq. 5 then Eq. 2, and Eq. 2 alone) agrees bit for bit."""
    cnf = gen.planted_ksat(700, 2800, 3, seed=5)
    for mode in (tsat.MODE_MEAN, tsat.MODE_NONE):
        s = tsat.Solver(params=tsat.default_params(norm_mode=mode))
        try:
            s.load(cnf)
            for N, seed in ((100, 7), (64, 2**40 + 3), (256, 1001)):
                s.init_batch(N, seed=seed)
                th = s.get_logits()
                ref = orc.init_normal(700, N, seed)
                assert ulp_close(th, ref).all()
                assert (th != ref).sum() <= 2
                b_ref, _ = orc.binarize(ref.astype(np.float64), mode)
                assert np.array_equal(tsat.unpack_bits(s.get_bits(), N), b_ref)
        finally:
            s.close()


@pytest.mark.parametrize("mode", [tsat.MODE_NONE, tsat.MODE_MEAN])
def test_proposal_init_vs_oracle(mode):
    s = solver_or_skip()
    try:
        s2 = tsat.Solver(params=tsat.default_params(norm_mode=mode))
    finally:
        s.close()
    cnf = gen.planted_ksat(900, 3600, 3, seed=6)
    s2.load(cnf)
    g = np.random.default_rng(1)
    p = g.uniform(0, 1, 900).astype(np.float32)
    p[:30] = 0.0
    p[30:60] = 1.0
    p[60:70] = np.nan
    p[70:80] = 1.5
    p[80:90] = -0.5
    for N, seed in ((100, 9), (32, 123456789)):
        s2.init_from_proposal(N, seed=seed, p_true=p)
        th = s2.get_logits()
        ref = orc.init_proposal(p, N, seed, mode)
        assert np.array_equal(th > 0, ref > 0)
        assert ulp_close(th, ref).all()
        # the solver's bits are the drawn ones (Eq. 5 then Eq. 2 reproduce them)
        bits = tsat.unpack_bits(s2.get_bits(), N)
        assert np.array_equal(bits, (ref > 0).astype(np.uint8))
    s2.close()


# --------------------------------------------------------------------------
# the network
# --------------------------------------------------------------------------

def rand_params(seed):
    g = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    p["b1"] = g.normal(0, 0.1, 128)
    p["b2"] = g.normal(0, 0.1, 128)
    p["b3"] = np.array([0.2])
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def rand_rows(seed, B, params, scale=1.0):
    """Feature-like rows (FP32), with the rows the oracle flags as fragile redrawn."""
    g = np.random.default_rng(seed)
    X = (g.normal(0, scale, (B, 16))).astype(np.float32)
    for _ in range(50):
        bad = mlp.fragile_rows(params, X.astype(np.float64))
        if not bad.any():
            break
        X[bad] = g.normal(0, scale, (int(bad.sum()), 16)).astype(np.float32)
    assert not mlp.fragile_rows(params, X.astype(np.float64)).any()
    return X


def out_scale(params, X):
    f = mlp.forward(params, X.astype(np.float64))
    s2 = f["h1q"] @ np.abs(f["W2q"]) + np.abs(params["b2"])
    return s2 @ np.abs(f["w3q"]) + abs(params["b3"][0])


@pytest.mark.parametrize("B", [1, 37, 64, 1000, 5003])
def test_forward_vs_oracle(torch, B):
    params = rand_params(31)
    net = tsat.Mlp(mlp.flatten(params).astype(np.float32))
    X = rand_rows(32 + B, B, params)
    Xd = torch.from_numpy(X).cuda()
    lo = torch.full((B + 5,), 7.0, device="cuda")
    pr = torch.full((B + 5,), 7.0, device="cuda")
    net.forward_dev(Xd.data_ptr(), B, lo.data_ptr(), pr.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = lo.cpu().numpy()
    ref = mlp.forward(params, X.astype(np.float64))["out"]
    rel = np.abs(got[:B] - ref) / out_scale(params, X)
    assert rel.max() <= 2e-5  # the worst-case bound of the FP32 sums
    assert np.median(rel) <= 1e-6  # typical rounding, far below it
    assert (got[B:] == 7.0).all()  # nothing written past B
    np.testing.assert_allclose(pr.cpu().numpy()[:B], mlp.sigmoid(got[:B].astype(np.float64)), rtol=2e-6, atol=1e-7)
    net.close()


def grad_check(net, params, X, y, w, torch):
    B = X.shape[0]
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    wd = None if w is None else torch.from_numpy(w.astype(np.float32)).cuda()
    net.train_step_dev(Xd.data_ptr(), yd.data_ptr(), None if wd is None else wd.data_ptr(), B, 0.0,
                       torch.cuda.current_stream().cuda_stream)
    g, loss = net.get_grad()
    rl, rg, _ = mlp.loss_and_grad(params, X.astype(np.float64), y, w)
    bound = mlp.flatten(mlp.abs_grad_bound(params, X.astype(np.float64), y, w))
    err = np.abs(g - mlp.flatten(rg))
    assert (err <= 1e-5 * bound + 1e-12).all(), (np.argmax(err / (bound + 1e-30)), (err / (bound + 1e-30)).max())
    assert abs(loss - rl) <= 1e-5 * abs(rl)
    return g


@pytest.mark.parametrize("B,weighted", [(1, False), (100, True), (4096, False), (20011, True)])
def test_gradient_vs_oracle(torch, B, weighted):
    params = rand_params(41)
    net = tsat.Mlp(mlp.flatten(params).astype(np.float32))
    X = rand_rows(42 + B, B, params)
    g = np.random.default_rng(B)
    y = (g.random(B) < 0.5).astype(np.float64)
    w = g.uniform(0.2, 3.0, B) if weighted else None
    grad_check(net, params, X, y, w, torch)
    net.close()


def test_adam_steps_vs_oracle(torch):
    params = rand_params(51)
    net = tsat.Mlp(mlp.flatten(params).astype(np.float32))
    B = 3000
    X = rand_rows(52, B, params)
    y = (np.random.default_rng(53).random(B) < 0.3).astype(np.float64)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    st = torch.cuda.current_stream().cuda_stream
    p_ref = {k: v.copy() for k, v in params.items()}
    m = {k: np.zeros_like(v) for k, v in params.items()}
    v = {k: np.zeros_like(x) for k, x in params.items()}
    for t in (1, 2, 3):
        net.train_step_dev(Xd.data_ptr(), yd.data_ptr(), None, B, 1e-3, st)
        g, _ = net.get_grad()
        # Adam from the GPU's own gradient: isolates the update arithmetic
        mlp.adam(p_ref, mlp.unflatten(g.astype(np.float64)), m, v, t, 1e-3)
        got = net.get_params()
        ref = mlp.flatten(p_ref)
        assert (np.abs(got - ref) <= 1e-6 * np.maximum(1.0, np.abs(ref))).all(), np.abs(got - ref).max()
        p_ref = mlp.unflatten(got.astype(np.float64))  # continue from the GPU's parameters
    assert net.step_count() == 3
    # the rounded operands follow the updated parameters: forward parity again
    Xf = rand_rows(54, 777, p_ref)
    Xfd = torch.from_numpy(Xf).cuda()
    lo = torch.empty(777, device="cuda")
    net.forward_dev(Xfd.data_ptr(), 777, lo.data_ptr(), None, st)
    torch.cuda.synchronize()
    ref = mlp.forward(p_ref, Xf.astype(np.float64))["out"]
    assert (np.abs(lo.cpu().numpy() - ref) <= 2e-5 * out_scale(p_ref, Xf)).all()
    net.close()


def test_training_reduces_loss_on_a_learnable_target(torch):
    """Labels from a fixed rule of the features: GPU Adam steps lower the loss."""
    params = mlp.init_params(61)
    net = tsat.Mlp(mlp.flatten(params).astype(np.float32))
    g = np.random.default_rng(62)
    B = 8192
    X = g.normal(0, 1, (B, 16)).astype(np.float32)
    y = ((X[:, 2] + 0.5 * X[:, 4] - 0.3 * X[:, 9]) > 0).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    st = torch.cuda.current_stream().cuda_stream
    net.train_step_dev(Xd.data_ptr(), yd.data_ptr(), None, B, 0.0, st)
    _, l0 = net.get_grad()
    for _ in range(300):
        net.train_step_dev(Xd.data_ptr(), yd.data_ptr(), None, B, 3e-3, st)
    net.train_step_dev(Xd.data_ptr(), yd.data_ptr(), None, B, 0.0, st)
    _, l1 = net.get_grad()
    assert l1 < 0.25 * l0, (l0, l1)
    # and the trained parameters still match the oracle's forward pass
    pt = mlp.unflatten(net.get_params().astype(np.float64))
    Xs = rand_rows(63, 500, pt)
    lo = torch.empty(500, device="cuda")
    net.forward_dev(torch.from_numpy(Xs).cuda().data_ptr(), 500, lo.data_ptr(), None, st)
    torch.cuda.synchronize()
    ref = mlp.forward(pt, Xs.astype(np.float64))["out"]
    assert (np.abs(lo.cpu().numpy() - ref) <= 2e-5 * out_scale(pt, Xs)).all()
    net.close()


def test_propose_then_init(solver, torch):
    cnf = gen.planted_ksat(3000, 12300, 3, seed=71)
    solver.load(cnf)
    params = rand_params(72)
    net = tsat.Mlp(mlp.flatten(params).astype(np.float32))
    p = solver.propose(net)
    # p is the network applied to the solver's own features
    X = solver.get_features()
    Xd = torch.from_numpy(X).cuda()
    pr = torch.empty(3000, device="cuda")
    net.forward_dev(Xd.data_ptr(), 3000, None, pr.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(pr.cpu().numpy(), p)
    assert ((p > 0) & (p < 1)).all()
    solver.init_from_proposal(96, seed=5)
    th = solver.get_logits()
    ref = orc.init_proposal(p, 96, 5, tsat.MODE_MEAN)
    assert np.array_equal(th > 0, ref > 0) and ulp_close(th, ref).all()
    net.close()


def test_learned_api_errors(solver):
    with pytest.raises(tsat.TsatError) as e:
        solver.init_from_proposal(8, seed=1)
    assert e.value.code == tsat.E_STATE
    cnf = gen.planted_ksat(50, 200, 3, seed=1)
    solver.load(cnf)
    with pytest.raises(tsat.TsatError) as e:
        solver.init_from_proposal(8, seed=1)
    assert e.value.code == tsat.E_STATE
    with pytest.raises(tsat.TsatError) as e:
        solver.init_from_proposal(2000, seed=1, p_true=np.full(50, 0.5, np.float32))
    assert e.value.code == tsat.E_ARG
    bad = np.zeros(tsat.MLP_NUM_PARAMS, np.float32)
    bad[5] = np.nan
    with pytest.raises(tsat.TsatError) as e:
        tsat.Mlp(bad)
    assert e.value.code == tsat.E_ARG
    net = tsat.Mlp(np.zeros(tsat.MLP_NUM_PARAMS, np.float32))
    with pytest.raises(tsat.TsatError) as e:
        net.get_grad()
    assert e.value.code == tsat.E_STATE
    net.close()
