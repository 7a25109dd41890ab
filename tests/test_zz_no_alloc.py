"""The allocation-free forward entry point (tsat_fwd_dev_noalloc) against the
allocating one (tsat_fwd_dev) and the oracle, through the C-ABI.

Both calls run the same forward kernels and the same SmoothMin kernel on the
same bits, so S and the histogram must agree bitwise; the histogram is
integer work and must also equal the oracle's exactly.  Every case makes two
calls in a row on the shared fixed scratch array, the second with fewer
candidates than the first, so a stale accumulator or unit table would show.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("torch sees no GPU")
    yield torch


def _mixed_cnf():
    """Widths 1-3 and 5-12 (every forward kernel), duplicates and a tautology."""
    g = np.random.default_rng(11)
    V = 400
    clauses = [[5], [-9]]
    for k in list(range(2, 4)) * 300 + list(range(5, 13)) * 30:
        vs = g.choice(V, size=k, replace=False) + 1
        clauses.append(list(np.where(g.random(k) < 0.5, vs, -vs)))
    clauses.append([3, -3, 7])
    clauses.append([4, 4, -8])
    return V, clauses


def _bits_with_garbage_pad(b, torch):
    """Packed value rows; the unused high bits of the last word are random
    (both entry points must ignore them)."""
    V, N = b.shape
    packed = tsat.pack_bits(b)
    if N % 64:
        g = np.random.default_rng(N)
        junk = g.integers(0, 2**63, size=V, dtype=np.uint64) << np.uint64(N % 64)
        packed[:, -1] |= junk
    return torch.tensor(packed.view(np.int64), device="cuda")


def _compare(torch, s, ocnf, V, K1, N, seed, tau):
    b = (np.random.default_rng(seed).random((V, N)) < 0.5).astype(np.uint8)
    bits = _bits_with_garbage_pad(b, torch)
    stream = torch.cuda.current_stream().cuda_stream
    S_ref = torch.empty(N, dtype=torch.float32, device="cuda")
    H_ref = torch.empty((N, K1), dtype=torch.int32, device="cuda")
    s.fwd_dev(bits.data_ptr(), N, tau, S_ref.data_ptr(), H_ref.data_ptr(), stream)
    S = torch.full((N,), float("nan"), dtype=torch.float32, device="cuda")
    H = torch.full((N, K1), -1, dtype=torch.int32, device="cuda")
    s.fwd_dev_noalloc(bits.data_ptr(), N, tau, S.data_ptr(), H.data_ptr(), stream)
    torch.cuda.synchronize()
    H_np = H.cpu().numpy().astype(np.int64)
    assert np.array_equal(H_np, H_ref.cpu().numpy().astype(np.int64))
    assert np.array_equal(S.cpu().numpy().view(np.uint32), S_ref.cpu().numpy().view(np.uint32))
    assert np.array_equal(H_np, orc.histogram(ocnf, b))


@pytest.mark.parametrize("case", ["planted3", "mixed"])
def test_noalloc_forward_matches_allocating_forward(env, case):
    torch = env
    s = tsat.Solver()
    try:
        if case == "planted3":
            cnf = gen.planted_ksat(300, 1200, 3, seed=5)
            s.load(cnf)
            ocnf = orc.Cnf.from_gen(cnf)
            V = 300
        else:
            V, clauses = _mixed_cnf()
            cnf = gen.CNF.from_clauses(V, clauses)
            s.load(cnf)
            ocnf = orc.Cnf.from_gen(cnf)
        K1 = s.max_width + 1
        # two calls in a row on the shared array, the second with fewer candidates
        for N, seed, tau in ((200, 1, 1.0), (37, 2, 0.5)):
            _compare(torch, s, ocnf, V, K1, N, seed, tau)
    finally:
        s.close()


def test_noalloc_forward_shared_between_solvers(env):
    """Two solvers on one GPU share the fixed array; calls are ordered on one
    stream, so each sees only its own results."""
    torch = env
    a, b = tsat.Solver(), tsat.Solver()
    try:
        ca = gen.planted_ksat(250, 1000, 3, seed=8)
        cb = gen.planted_ksat(120, 500, 3, seed=9)
        a.load(ca)
        b.load(cb)
        _compare(torch, a, orc.Cnf.from_gen(ca), 250, a.max_width + 1, 256, 3, 1.0)
        _compare(torch, b, orc.Cnf.from_gen(cb), 120, b.max_width + 1, 64, 4, 2.0)
        _compare(torch, a, orc.Cnf.from_gen(ca), 250, a.max_width + 1, 1, 5, 1.0)
    finally:
        a.close()
        b.close()


def test_noalloc_forward_rejects_bad_sizes(env):
    torch = env
    s = tsat.Solver()
    try:
        s.load(gen.planted_ksat(50, 200, 3, seed=2))
        bits = torch.zeros((50, 32), dtype=torch.int64, device="cuda")
        out = torch.empty(2048, dtype=torch.float32, device="cuda")
        for n in (0, tsat.MAX_STEP_N + 1):
            with pytest.raises(tsat.TsatError) as e:
                s.fwd_dev_noalloc(bits.data_ptr(), n, 1.0, out.data_ptr(), None)
            assert e.value.code == tsat.E_ARG
        with pytest.raises(tsat.TsatError) as e:
            s.fwd_dev_noalloc(bits.data_ptr(), 8, -1.0, out.data_ptr(), None)
        assert e.value.code == tsat.E_ARG
    finally:
        s.close()
