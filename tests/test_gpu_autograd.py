"""torch.autograd.Function over the HIP forward/adjoint vs the FP64 oracle and
finite differences of the relaxed objective (Eq. 3/4 on real-valued x)."""
import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

from parity_util import (TOL_GRAD, abs_adjoint, grad_bound, make_state, solver_or_skip, sub_cnf)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    s = solver_or_skip()
    if not torch.cuda.is_available():
        pytest.skip("torch sees no GPU")
    from paper_2511_07737_amd import autograd

    yield torch, s, autograd
    s.close()


def mixed_cnf():
    s = gen.structured(640, 3000, seed=4)
    clauses = [list(s.clause(c)) for c in range(s.num_clauses)] + [[5, 5, -7], [9, -9], [13]]
    return gen.CNF.from_clauses(645, clauses)


def test_forward_and_backward_vs_oracle(env):
    torch, solver, ag = env
    cnf = mixed_cnf()
    solver.load(cnf)
    oc = orc.Cnf.from_gen(cnf)
    N = 100
    rng = np.random.default_rng(5)
    b = rng.integers(0, 2, size=(cnf.num_vars, N)).astype(np.uint8)
    for tau in (0.5, 1.0, 2.0):
        print(f"[autograd] tau={tau}", flush=True)
        A = torch.tensor(b, dtype=torch.float32, device="cuda", requires_grad=True)
        S = ag.smoothmin_sat(A, solver, tau)
        H = orc.histogram(oc, b)
        w = rng.normal(size=N)
        S_ref, table, _ = orc.smoothmin(H, tau, w)
        assert np.allclose(S.detach().cpu().numpy(), S_ref, rtol=1e-6, atol=1e-6)
        (S * torch.tensor(w, dtype=torch.float32, device="cuda")).sum().backward()
        U = A.grad.cpu().numpy()
        U_ref = orc.adjoint(oc, b, table)
        aU = abs_adjoint(oc, b, table)
        # the upstream gradient is rounded to FP32 on the GPU: add its rounding
        assert (np.abs(U - U_ref) <= TOL_GRAD * aU + 1e-7 * aU + 1e-30).all(), np.abs(U - U_ref).max()


def fd_coords(oc, b, coords, w, tau, h=1e-3):
    """Central differences of sum_i w_i S~_i(x) at the binary point b."""
    x = b.astype(np.float64)
    return np.array([w[i] * orc.relaxed_fd(oc, x, v, i, h, tau) for v, i in coords])


def test_backward_vs_finite_differences(env):
    torch, solver, ag = env
    cnf = gen.planted_ksat(300, 1230, 3, seed=8)
    solver.load(cnf)
    oc = orc.Cnf.from_gen(cnf)
    N = 64
    rng = np.random.default_rng(9)
    b = rng.integers(0, 2, size=(300, N)).astype(np.uint8)
    w = rng.normal(size=N)
    A = torch.tensor(b, dtype=torch.float32, device="cuda", requires_grad=True)
    (ag.smoothmin_sat(A, solver, 1.0) * torch.tensor(w, dtype=torch.float32, device="cuda")).sum().backward()
    U = A.grad.cpu().numpy()
    coords = [(int(v), int(i)) for v, i in zip(rng.integers(0, 300, 200), rng.integers(0, N, 200))]
    fd = fd_coords(oc, b, coords, w, 1.0)
    H = orc.histogram(oc, b)
    _, table, _ = orc.smoothmin(H, 1.0, w)
    U_ref = orc.adjoint(oc, b, table)
    ref = np.array([U_ref[v, i] for v, i in coords])
    got = np.array([U[v, i] for v, i in coords])
    fd_err = np.abs(fd - ref)  # truncation error of the central difference (h = 1e-3)
    assert fd_err.max() <= 1e-6 * np.abs(ref).max() + 1e-9
    assert (np.abs(got - fd) <= 2 * fd_err + 1e-5 * np.abs(ref).max()).all()


@pytest.mark.timeout(600)
def test_structured_config_fd_and_oracle(env):
    """The structured configuration at full size through the autograd Function:
    sampled coordinates against central differences (h = 1e-3, FP64) of the
    relaxed objective and against the oracle's adjoint."""
    torch, solver, ag = env
    cnf = gen.structured(500_000, 2_500_000, seed=2)
    print("[autograd] structured config loaded", flush=True)
    solver.load(cnf)
    N = 128
    th, _, _ = make_state(cnf.num_vars, N, 1002, t_moments=False)
    b = (th > 0).astype(np.uint8)
    rng = np.random.default_rng(2)
    w = -np.ones(N)  # the loss of Eq. 3
    A = torch.tensor(b, dtype=torch.float32, device="cuda", requires_grad=True)
    (-ag.smoothmin_sat(A, solver, 1.0).sum()).backward()
    U = A.grad.cpu().numpy()
    oc = orc.Cnf.from_gen(cnf)
    H = orc.histogram(oc, b)
    _, table, _ = orc.smoothmin(H, 1.0)
    deg = np.bincount(np.abs(cnf.lits) - 1, minlength=cnf.num_vars)
    pick = np.unique(np.concatenate([rng.choice(cnf.num_vars, 24, replace=False), np.argsort(deg)[-2:]]))
    osub = orc.Cnf.from_gen(sub_cnf(cnf, pick))
    U_ref = orc.adjoint(osub, b, table)[pick]
    aU = abs_adjoint(osub, b, table)[pick]
    assert (np.abs(U[pick] - U_ref) <= TOL_GRAD * aU + 1e-30).all()
    coords = [(int(v), int(rng.integers(0, N))) for v in pick[:12]]
    got = np.array([U[v, i] for v, i in coords])
    ref = np.array([U_ref[list(pick).index(v), i] for v, i in coords])
    scale = np.abs(ref).max()
    # h = 1e-3 (the configuration's step): the GPU is as close to the central
    # difference as the FP64 oracle is, up to 1e-5 of the gradient scale
    fd = fd_coords(oc, b, coords, w, 1.0, h=1e-3)
    fd_err = np.abs(fd - ref)
    assert fd_err.max() <= 1e-5 * scale  # O(h^2) truncation of a smooth objective
    assert (np.abs(got - fd) <= fd_err + 1e-5 * scale).all()


def _chain_reference(oc, th, mode, tau=1.0):
    """Oracle loss and dL/dtheta of theta -> Eq. 5 -> Eq. 2 -> Eq. 1 -> Eq. 4 -> Eq. 3,
    and the error scale a_g of the gradient."""
    p = orc.default_params(mode=mode, tau=tau)
    ref = orc.step(oc, th.astype(np.float64), np.zeros_like(th, np.float64), np.zeros_like(th, np.float64), 0, p)
    b, mu = orc.binarize(th.astype(np.float64), mode)
    _, table, _ = orc.smoothmin(orc.histogram(oc, b), tau)
    aU = abs_adjoint(oc, b, table)
    ag = grad_bound(aU, th, mu if mode == orc.MODE_MEAN else np.ones_like(mu), ref["g"])
    return ref, b, mu, ag


@pytest.mark.parametrize("normalize", [True, False])
def test_full_chain_gradient(env, normalize):
    """theta -> Eq. 5 -> STE binarize -> layer -> Eq. 3 in one Function (loss and
    its fused backward in the library): loss and theta.grad vs the oracle."""
    torch, solver, ag = env
    cnf = gen.planted_ksat(200, 800, 3, seed=1)
    solver.load(cnf)
    oc = orc.Cnf.from_gen(cnf)
    th, _, _ = make_state(200, 64, 1001, t_moments=False, min_abs_mu=1e-2)
    mode = orc.MODE_MEAN if normalize else orc.MODE_NONE
    T = torch.tensor(th, device="cuda", requires_grad=True)
    loss = ag.loss_of(T, solver, 1.0, normalize=normalize)
    (2.5 * loss).backward()  # an upstream gradient other than 1
    ref, _, _, a_g = _chain_reference(oc, th, mode)
    assert abs(loss.item() - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    g = T.grad.cpu().numpy()
    assert (np.abs(g - 2.5 * ref["g"]) <= TOL_GRAD * 2.5 * a_g + 1e-30).all(), np.abs(g - 2.5 * ref["g"]).max()


@pytest.mark.parametrize("normalize", [True, False])
def test_composed_chain_gradient(env, normalize):
    """The same chain composed from its pieces: binarize (Eq. 5, Eq. 2 with the
    STE and the Eq. 5 backward) feeding the SmoothMin layer; the loss sum is
    formed by the test."""
    torch, solver, ag = env
    cnf = mixed_cnf()
    solver.load(cnf)
    oc = orc.Cnf.from_gen(cnf)
    th, _, _ = make_state(cnf.num_vars, 100, 1003, t_moments=False, min_abs_mu=1e-2)
    mode = tsat.MODE_MEAN if normalize else tsat.MODE_NONE
    T = torch.tensor(th, device="cuda", requires_grad=True)
    A = ag.binarize(T, solver, mode)
    S = ag.smoothmin_sat(A, solver, 1.0)
    loss = -S.sum()
    loss.backward()
    ref, b, _, a_g = _chain_reference(oc, th, mode)
    assert np.array_equal(A.detach().cpu().numpy(), b.astype(np.float32))
    assert abs(loss.item() - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    g = T.grad.cpu().numpy()
    assert (np.abs(g - ref["g"]) <= TOL_GRAD * a_g + 1e-30).all(), np.abs(g - ref["g"]).max()


@pytest.mark.parametrize("N", [1, 64, 100, 256])
def test_binarize_and_norm_backward_dev(env, N):
    """The device-pointer Eq. 5 / Eq. 2 and Eq. 5 backward calls against the oracle:
    bits and 0/1 values exact, row means to FP64 rounding, g within 1e-5 of its
    term sizes; a zero-mean row takes the clamp."""
    torch, solver, _ = env
    cnf = gen.planted_ksat(300, 1200, 3, seed=5)
    solver.load(cnf)
    th, _, _ = make_state(300, N, 1100 + N, t_moments=False)
    if N > 1:
        th[7] = 0.0  # mean 0: clamped to +1e-12, every entry maps to 0
        th[8, :] = np.float32(0.5)
        th[8, 0] = np.float32(-0.5 * (N - 1))  # exact zero mean with nonzero entries
    rng = np.random.default_rng(N)
    dA = rng.standard_normal(size=(300, N)).astype(np.float32)
    W = (N + 63) // 64
    stream = torch.cuda.current_stream().cuda_stream
    T = torch.tensor(th, device="cuda")
    for mode in (tsat.MODE_MEAN, tsat.MODE_NONE):
        bits = torch.empty((300, W), dtype=torch.int64, device="cuda")
        A = torch.empty((300, N), dtype=torch.float32, device="cuda")
        mu = torch.empty(300, dtype=torch.float64, device="cuda")
        solver.binarize_dev(T.data_ptr(), N, mode, bits.data_ptr(), A.data_ptr(), mu.data_ptr(), stream)
        b_ref, mu_ref = orc.binarize(th.astype(np.float64), mode)
        got_bits = tsat.unpack_bits(bits.cpu().numpy().view(np.uint64), N)
        assert np.array_equal(got_bits, b_ref)
        assert np.array_equal(A.cpu().numpy(), b_ref.astype(np.float32))
        if mode == tsat.MODE_MEAN:
            assert np.allclose(mu.cpu().numpy(), th.astype(np.float64).mean(axis=1), rtol=1e-12, atol=1e-15)
        g = torch.empty_like(T)
        D = torch.tensor(dA, device="cuda")
        solver.norm_backward_dev(T.data_ptr(), D.data_ptr(), N, mode, g.data_ptr(), stream)
        g_ref = orc.norm_backward(th.astype(np.float64), dA.astype(np.float64), mode)
        if mode == tsat.MODE_MEAN:
            m = th.astype(np.float64).mean(axis=1, keepdims=True)
            clamped = np.abs(m) < 1e-12
            m = np.where(clamped, np.where(m >= 0, 1e-12, -1e-12), m)
            corr = np.where(clamped, 0.0, (np.abs(dA) * np.abs(th)).sum(axis=1, keepdims=True) / (N * m * m))
            scale = np.abs(dA) / np.abs(m) + corr + np.abs(g_ref)
        else:
            scale = np.abs(g_ref)
        assert (np.abs(g.cpu().numpy() - g_ref) <= 1e-5 * scale + 1e-30).all()


def test_device_calls_reject_bad_arguments(env):
    torch, solver, _ = env
    cnf = gen.planted_ksat(50, 200, 3, seed=2)
    solver.load(cnf)
    T = torch.zeros((50, 8), dtype=torch.float32, device="cuda")
    out = torch.empty((), dtype=torch.float32, device="cuda")
    with pytest.raises(tsat.TsatError) as e:
        solver.loss_dev(T.data_ptr(), 8, -1.0, tsat.MODE_MEAN, out.data_ptr(), None, None)
    assert e.value.code == tsat.E_ARG
    with pytest.raises(tsat.TsatError) as e:
        solver.binarize_dev(T.data_ptr(), 8, 5, None, None, None)
    assert e.value.code == tsat.E_ARG
    with pytest.raises(tsat.TsatError) as e:
        solver.loss_backward_dev(T.data_ptr(), 0, 1.0, tsat.MODE_MEAN, None, T.data_ptr(), None)
    assert e.value.code == tsat.E_ARG
