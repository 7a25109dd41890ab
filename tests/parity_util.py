"""Helpers shared by the GPU parity tests: seeded states, oracle references and
the error bounds the comparisons use.

Tolerances follow from the arithmetic of the GPU path:
  * bits, histograms, satisfied counts, verdicts: integer work, compared exactly;
  * U: the GPU sums FP32-rounded dL/dR table entries in FP64, so its error is
    at most 2^-24 of a_U = sum over occurrences of |table[R]|; the test allows
    1e-5 * a_U (the gradient tolerance of the method's FP32 path);
  * g (Eq. 5 backward, FP64 on the GPU): 1e-5 * a_g with
    a_g = a_U / |mu| + sum_k |theta_k| a_U,k / (N mu^2) + |g|;
  * AdamW (FP32 with FP64-derived scalars), given the GPU's own g: a few FP32
    ulps of each term, allowed 2e-6 of the sum of term magnitudes.
"""
from __future__ import annotations

import numpy as np

import oracle as orc
from paper_2511_07737_amd import gen, tsat

TOL_GRAD = 1e-5
TOL_ADAM = 2e-6


def solver_or_skip():
    import pytest

    try:
        return tsat.Solver()
    except tsat.TsatError as e:
        if e.code == tsat.E_HIP and "no HIP device" in str(e):
            pytest.skip("no GPU visible")
        raise


def make_state(V, N, seed, t_moments=True, min_abs_mu=1e-3):
    """theta ~ N(0,1) float32 with rows of tiny mean redrawn; m, v small."""
    th = gen.normal_logits(V, N, seed)
    g = gen.rng(seed + 77)
    for _ in range(20):
        mu = th.astype(np.float64).mean(axis=1)
        bad = np.abs(mu) < min_abs_mu
        if not bad.any():
            break
        th[bad] = g.standard_normal(size=(int(bad.sum()), N), dtype=np.float32)
    if not t_moments:
        return th, np.zeros_like(th), np.zeros_like(th)
    m = (g.standard_normal(size=(V, N), dtype=np.float32) * 0.05).astype(np.float32)
    v = (np.abs(g.standard_normal(size=(V, N), dtype=np.float32)) * 0.01 + 1e-6).astype(np.float32)
    return th, m, v


def abs_adjoint(cnf_o: orc.Cnf, b: np.ndarray, table: np.ndarray) -> np.ndarray:
    """a_U[v][i] = sum over clauses c containing v of |table[i][R_ci]| (error scale of U)."""
    off, lit = cnf_o.clauses()
    R = orc.result_matrix(cnf_o, b)  # [C][N]
    N = b.shape[1]
    A = np.zeros((cnf_o.V, N), dtype=np.float64)
    if cnf_o.L == 0:
        return A
    cid = np.repeat(np.arange(cnf_o.C), np.diff(off))
    var = np.abs(lit) - 1
    vals = np.abs(table[np.arange(N)[None, :], R[cid]])  # [L][N]
    np.add.at(A, var, vals)
    return A


def grad_bound(aU, theta, mu, g):
    N = theta.shape[1]
    th = theta.astype(np.float64)
    mu = mu[:, None]
    s = (np.abs(th) * aU).sum(axis=1, keepdims=True)
    return aU / np.abs(mu) + s / (N * mu * mu) + np.abs(g)


def sub_cnf(cnf: gen.CNF, vars0: np.ndarray) -> gen.CNF:
    """Clauses of cnf that contain any of the 0-based variables vars0 (same V)."""
    sel = np.zeros(cnf.num_vars, dtype=bool)
    sel[vars0] = True
    w = cnf.widths()
    cid = np.repeat(np.arange(cnf.num_clauses), w)
    hit = np.zeros(cnf.num_clauses, dtype=bool)
    hit[cid[sel[np.abs(cnf.lits) - 1]]] = True
    keep = np.nonzero(hit)[0]
    clauses = [cnf.clause(c) for c in keep]
    return gen.CNF.from_clauses(cnf.num_vars, clauses)


def adam_reference(theta, m, v, g, t, p, count=None):
    """Oracle AdamW on float64 copies; t is the 0-based iteration index, count
    the bias-correction count (t + 1 from a fresh optimizer)."""
    th = theta.astype(np.float64).copy()
    mm = m.astype(np.float64).copy()
    vv = v.astype(np.float64).copy()
    lr = orc.lr(t, orc.default_params(lr0=p.lr0, decay=p.lr_decay, every=p.decay_every,
                                      restart=p.restart_every, lr_min=p.lr_min))
    orc.adamw(th, mm, vv, g.astype(np.float64), lr, t + 1 if count is None else count, p.beta1, p.beta2, p.eps,
              p.weight_decay)
    return th, mm, vv, lr


def adam_bounds(theta, m, v, g, t, p, lr, v_new, count=None):
    th = np.abs(theta.astype(np.float64))
    g64 = g.astype(np.float64)
    n = t + 1 if count is None else count
    bc1 = 1 - p.beta1 ** n
    bc2 = 1 - p.beta2 ** n
    m_abs = p.beta1 * np.abs(m) + (1 - p.beta1) * np.abs(g64)
    v_abs = p.beta2 * np.abs(v) + (1 - p.beta2) * g64 * g64
    step = (lr / bc1) * m_abs / (np.sqrt(np.abs(v_new)) / np.sqrt(bc2) + p.eps)
    return th * (1 - lr * p.weight_decay) + step, m_abs, v_abs


def oparams(p):
    return orc.default_params(tau=p.tau, lr0=p.lr0, decay=p.lr_decay, lr_min=p.lr_min, beta1=p.beta1,
                              beta2=p.beta2, eps=p.eps, weight_decay=p.weight_decay, every=p.decay_every,
                              restart=p.restart_every, mode=p.norm_mode)


def one_step_parity(solver, cnf, N, seed, t, p=None, state=None, check_bits_rows=True):
    """Full element-by-element parity of one iteration."""
    p = p or tsat.default_params()
    print(f"[parity] V={cnf.num_vars} C={cnf.num_clauses} N={N} seed={seed} t={t} tau={p.tau} mode={p.norm_mode}",
          flush=True)
    solver.load(cnf)
    th, m, v = state if state is not None else make_state(cnf.num_vars, N, seed)
    solver.init_batch(N, init_logits=th)
    solver.set_state(th, m, v, t)
    oc = orc.Cnf.from_gen(cnf)
    # forward: bits (of the call's normalization mode), histogram, loss
    hist, S, loss = solver.eval(p)
    b_ref, mu = orc.binarize(th.astype(np.float64), p.norm_mode)
    b_gpu = tsat.unpack_bits(solver.get_bits(), N)
    assert np.array_equal(b_gpu, b_ref)
    H_ref = orc.histogram(oc, b_ref)
    assert hist.shape == H_ref.shape and np.array_equal(hist.astype(np.int64), H_ref)
    S_ref, table, loss_ref = orc.smoothmin(H_ref, p.tau)
    assert np.allclose(S, S_ref, rtol=1e-12, atol=1e-12)
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-12
    sat, ok = solver.check()
    sat_ref, ok_ref = orc.check(oc, b_ref)
    assert np.array_equal(sat, sat_ref) and np.array_equal(ok, ok_ref)
    # backward
    U_gpu, g_gpu = solver.get_grad(p)
    U_ref = orc.adjoint(oc, b_ref, table)
    aU = abs_adjoint(oc, b_ref, table)
    assert (np.abs(U_gpu - U_ref) <= TOL_GRAD * aU + 1e-30).all(), np.abs(U_gpu - U_ref).max()
    g_ref = orc.norm_backward(th.astype(np.float64), U_ref, p.norm_mode)
    ag = grad_bound(aU, th, mu, g_ref) if p.norm_mode == orc.MODE_MEAN else aU + np.abs(g_ref)
    assert (np.abs(g_gpu - g_ref) <= TOL_GRAD * ag + 1e-30).all(), np.abs(g_gpu - g_ref).max()
    # update (stage 2: the oracle optimizer applied to the GPU's gradient)
    rep = solver.step(1, params=p)
    assert rep.steps_done == 1 and rep.next_step == t + 1
    assert abs(rep.loss - loss_ref) <= 1e-5 * abs(loss_ref) + 1e-12
    th2, m2, v2, t2 = solver.get_state()
    assert t2 == t + 1
    th_r, m_r, v_r, lr = adam_reference(th, m, v, g_gpu, t, p)
    bt, bm, bv = adam_bounds(th, m, v, g_gpu, t, p, lr, v_r)
    assert (np.abs(m2 - m_r) <= TOL_ADAM * bm + 1e-30).all()
    assert (np.abs(v2 - v_r) <= TOL_ADAM * bv + 1e-30).all()
    assert (np.abs(th2 - th_r) <= TOL_ADAM * bt + 1e-30).all(), np.abs(th2 - th_r).max()
    # re-binarization of the GPU's own new logits (exact)
    b2_ref, mu2 = orc.binarize(th2.astype(np.float64), p.norm_mode)
    if check_bits_rows:
        b2_gpu = tsat.unpack_bits(solver.get_bits(), N)
        assert np.array_equal(b2_gpu, b2_ref)
    return dict(U=U_gpu, g=g_gpu, table=table, H=H_ref)
