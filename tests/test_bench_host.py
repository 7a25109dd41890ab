"""Host-side parts of bench.py (no GPU): the all-threads CPU baseline runs
the same oracle routines on parts of the variables / candidates, so one
iteration must equal orc.step bit for bit; the byte models follow their
definitions."""
import numpy as np

import bench
import oracle as orc
from paper_2511_07737_amd import gen


def test_threaded_oracle_step_equals_oracle_step():
    cnf = gen.planted_ksat(400, 1700, 3, seed=3)
    oc = orc.Cnf.from_gen(cnf)
    N = 70
    th0 = gen.normal_logits(400, N, 5).astype(np.float64)
    a = [th0.copy(), np.zeros_like(th0), np.zeros_like(th0)]
    b = [th0.copy(), np.zeros_like(th0), np.zeros_like(th0)]
    for t in range(3):
        r = orc.step(oc, a[0], a[1], a[2], t)
        a = [r["theta"], r["m"], r["v"]]
        bench.oracle_step_threaded(oc, b[0], b[1], b[2], t, threads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_byte_models():
    cnf = gen.planted_ksat(1000, 4100, 3, seed=1)
    N = 256
    sb = bench.model_bytes(cnf, N)
    V, L = 1000, cnf.num_lits
    assert sb["fwd"] == 4 * L + V * N / 8
    assert sb["update"] == 4 * L + 2 * V * N / 8 + 24 * V * N
    assert sb["fwdbwd"] == 8 * L + V * N / 4 + 4 * V * N
    assert sb["step_fused_min"] == sb["fwd"] + sb["update"]
    imp = bench.implementation_bytes(cnf, N, True)
    assert imp["planes_write"] == cnf.num_clauses * 2 * 4 * 8
    mixed = gen.CNF.from_clauses(10, [[1, 2], [3, 4, 5], [1, 2, 3, 4, 5, 6]])
    assert bench.implementation_bytes(mixed, 64, True)["planes_write"] == (2 + 2 + 4) * 1 * 8
    assert bench.uses_clause_planes(cnf, N, 1) and not bench.uses_clause_planes(cnf, 257, 1)
