"""Clause-plane gather by 64-record windows (vector loads, bits transposed
across the wavefront) against the record-by-record scalar gather: the counts
are exact, so the two give the same results bit for bit, on the step, the
gradient and the adjoint, for every row width, with variables whose records
span several windows, chunks that cross instance boundaries, and instances
frozen while the others move on.  Rows of at most 32 candidates take the
two-variables-per-wave form of the window gather, which reads a clause's two
planes packed in one 8-byte word while the record gather reads them unpacked
(pairs that straddle instance boundaries, an odd last pair, one frozen
variable of a pair).
Oracle parity of the window gather itself comes from the parity tests, where
it is the default."""
import numpy as np
import pytest

from paper_2511_07737_amd import gen, tsat

from parity_util import solver_or_skip

pytestmark = pytest.mark.gpu


def run(cnfs, N, window, steps, params=None, stop=False, seed=5):
    s = solver_or_skip()
    s.load_batch(cnfs)
    s.set_launch_config(window_gather=window)
    assert s.launch_config().window_gather == window
    s.init_batch(N, seed=seed)
    rep = s.step(steps, params=params, stop_on_sat=stop)
    th, m, v, t = s.get_state()
    out = dict(theta=th, m=m, v=v, t=t, bits=s.get_bits(), steps=rep.steps_done)
    out["U"], out["g"] = s.get_grad(params)
    out["status"] = s.instance_status()
    out["witness"] = [s.get_witness_instance(j, c.num_vars) if x["first_sat_step"] >= 0 else None
                      for j, (x, c) in enumerate(zip(out["status"], cnfs))]
    s.close()
    return out


def assert_same(a, b):
    for k in ("theta", "m", "v", "bits", "U", "g"):
        assert np.array_equal(a[k], b[k]), k
    assert a["t"] == b["t"] and a["steps"] == b["steps"]
    for x, y in zip(a["status"], b["status"]):
        for k in ("first_sat_step", "first_converged_step", "frozen", "sat_candidate", "best_sat_count"):
            assert x[k] == y[k], k
    for wa, wb in zip(a["witness"], b["witness"]):
        assert (wa is None) == (wb is None)
        if wa is not None:
            assert np.array_equal(wa[0], wb[0]) and wa[1] == wb[1]


@pytest.mark.parametrize("k,N", [(3, 256), (3, 200), (3, 100), (3, 64), (3, 33), (3, 32), (3, 17), (3, 1),
                                 (2, 256), (2, 64), (2, 9)])
def test_window_gather_equals_record_gather(k, N):
    V = 1001
    cnf = gen.planted_ksat(V, int((4.0 if k == 3 else 1.5) * V), k, seed=40 + k)
    print(f"[window] k={k} N={N}", flush=True)
    for mode in (tsat.MODE_MEAN, tsat.MODE_NONE):
        p = tsat.default_params(norm_mode=mode, tau=2.0 if mode == tsat.MODE_NONE else 1.0)
        assert_same(run([cnf], N, 1, 23, params=p), run([cnf], N, 0, 23, params=p))


def hub_cnf():
    """3-SAT with a few variables in hundreds of clauses: their records run
    over several 64-record windows."""
    rng = np.random.default_rng(12)
    V = 600
    clauses = []
    for c in range(2400):
        vs = rng.choice(V, size=3, replace=False) + 1
        if c % 3 == 0:
            vs[0] = 1 + (c // 3) % 4  # variables 1..4 appear ~200 times each
            if vs[0] in vs[1:]:
                continue
        sg = rng.choice([-1, 1], size=3)
        clauses.append([int(x) for x in vs * sg])
    return gen.CNF.from_clauses(V, clauses)


@pytest.mark.parametrize("N", [256, 64])
def test_window_gather_long_records(N):
    cnf = hub_cnf()
    assert (np.diff(cnf.offsets) == 3).all()  # uniform width: the clause-plane path
    p = tsat.default_params()
    assert_same(run([cnf], N, 1, 15, params=p), run([cnf], N, 0, 15, params=p))


@pytest.mark.parametrize("N", [64, 20])
def test_window_gather_variables_without_occurrences(N):
    """Variables that occur in no clause (empty record ranges, also inside a
    window and at the ends of a chunk or pair) get U = 0 like in the record
    gather."""
    rng = np.random.default_rng(8)
    V = 300
    used = np.arange(1, V + 1)
    used = used[(used % 7 != 0) & (used > 5) & (used < V - 3)]
    clauses = []
    for _ in range(900):
        vs = rng.choice(used, size=3, replace=False)
        clauses.append([int(x) for x in vs * rng.choice([-1, 1], size=3)])
    cnf = gen.CNF.from_clauses(V, clauses)
    p = tsat.default_params()
    assert_same(run([cnf], N, 1, 12, params=p), run([cnf], N, 0, 12, params=p))


def test_window_gather_off_for_very_frequent_variables():
    """The window gather keeps per-sign counts in 16 bits; a store with a
    variable in 2^16 or more clauses of one sign takes the record gather
    (same results as asking for it)."""
    rng = np.random.default_rng(21)
    V, C = 4000, 66000
    others = rng.choice(np.arange(2, V + 1), size=(C, 2))
    same = others[:, 0] == others[:, 1]
    others[same, 1] = others[same, 0] % (V - 1) + 2  # another variable in 2..V
    sg = rng.choice([-1, 1], size=(C, 2))
    clauses = [[1, int(a), int(b)] for (a, b) in others * sg]  # variable 1 in every clause
    cnf = gen.CNF.from_clauses(V, clauses)
    p = tsat.default_params()
    assert_same(run([cnf], 64, 1, 6, params=p), run([cnf], 64, 0, 6, params=p))


def test_window_gather_batch_with_frozen_instances():
    """Odd instance sizes put chunk boundaries inside instances; the easy
    members freeze on a satisfying candidate while the hard ones go on."""
    sizes = [(201, 560, 3), (333, 1365, 3), (99, 260, 3), (150, 615, 3), (77, 200, 3), (1201, 4920, 3)]
    cnfs = [gen.planted_ksat(V, C, kk, seed=60 + j) for j, (V, C, kk) in enumerate(sizes)]
    p = tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)
    for N in (32, 128):
        a = run(cnfs, N, 1, 600, params=p, stop=True, seed=8)
        b = run(cnfs, N, 0, 600, params=p, stop=True, seed=8)
        assert any(x["frozen"] for x in a["status"]), "no member froze in 600 steps"
        assert_same(a, b)


def test_window_gather_adjoint_equals_record_gather():
    torch = pytest.importorskip("torch")
    s = solver_or_skip()
    if not torch.cuda.is_available():
        s.close()
        pytest.skip("torch sees no GPU")
    from paper_2511_07737_amd import autograd

    cnf = gen.planted_ksat(777, 3100, 3, seed=71)
    s.load(cnf)
    rng = np.random.default_rng(3)
    for N in (24, 190):
        b = rng.integers(0, 2, size=(cnf.num_vars, N)).astype(np.float32)
        w = torch.tensor(rng.normal(size=N), dtype=torch.float32, device="cuda")
        grads = []
        for window in (1, 0):
            s.set_launch_config(window_gather=window)
            A = torch.tensor(b, device="cuda", requires_grad=True)
            (autograd.smoothmin_sat(A, s, 1.5) * w).sum().backward()
            grads.append(A.grad.cpu().numpy())
        assert np.array_equal(grads[0], grads[1])
    s.close()


def test_autotune_tries_both_plane_gathers():
    s = solver_or_skip()
    s.load(gen.planted_ksat(3001, 12300, 3, seed=5))
    s.init_batch(96, seed=1)
    c, used = s.autotune(iters=2)
    assert c.window_gather in (0, 1) and c.clause_planes in (0, 1)
    # forward targets; blocks per CU with the planes on, by windows and by
    # records; without planes, with the three record groups
    assert used == 2 * (8 + 9 * 2 + 9 * 3)
    with pytest.raises(tsat.TsatError) as e:
        s.set_launch_config(window_gather=2)
    assert e.value.code == tsat.E_ARG
    s.close()
