"""The clause-major atomic-scatter adjoint (tsat_bwd_scatter_dev, the
comparison design) against the FP64 oracle and against the variable-major
gather (tsat_bwd_dev).  Its FP32 atomic additions come in no fixed order, so
each U entry is checked within (degree + 1) 2^-24 of a_U, the sum of its
terms' magnitudes (no more than the gradient tolerance here)."""
import numpy as np
import pytest

import oracle as orc
from paper_2511_07737_amd import gen, tsat

from parity_util import TOL_GRAD, abs_adjoint, solver_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("torch sees no GPU")
    s = solver_or_skip()
    yield torch, s
    s.close()


@pytest.mark.parametrize("kind,N", [("planted", 256), ("planted", 100), ("mixed", 64), ("mixed", 33)])
def test_scatter_adjoint_matches_oracle_and_gather(env, kind, N):
    torch, s = env
    if kind == "planted":
        cnf = gen.planted_ksat(900, 3690, 3, seed=21)
    else:
        g = np.random.default_rng(22)
        clauses = [list(int(x) * int(g.choice([-1, 1])) for x in g.choice(600, size=k, replace=False) + 1)
                   for k in [1, 2, 3, 4, 6, 9, 14, 20] * 40]
        cnf = gen.CNF.from_clauses(600, clauses)
    s.load(cnf)
    V = cnf.num_vars
    b = (np.random.default_rng(N).random((V, N)) < 0.5).astype(np.uint8)
    dS = np.random.default_rng(N + 1).standard_normal(N).astype(np.float32)
    bits = torch.tensor(tsat.pack_bits(b).view(np.int64), device="cuda")
    dSt = torch.tensor(dS, device="cuda")
    U1 = torch.empty((V, N), dtype=torch.float32, device="cuda")
    U2 = torch.full((V, N), float("nan"), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    s.bwd_dev(bits.data_ptr(), N, 1.0, dSt.data_ptr(), U1.data_ptr(), st)
    s.bwd_scatter_dev(bits.data_ptr(), N, 1.0, dSt.data_ptr(), U2.data_ptr(), st)
    torch.cuda.synchronize()
    oc = orc.Cnf.from_gen(cnf)
    _, table, _ = orc.smoothmin(orc.histogram(oc, b), 1.0, dS.astype(np.float64))
    U_ref = orc.adjoint(oc, b, table)
    aU = abs_adjoint(oc, b, table)
    deg = np.zeros(V)
    np.add.at(deg, np.abs(cnf.lits) - 1, 1)
    tol = np.minimum(TOL_GRAD, (deg[:, None] + 1) * 2.0**-24 + 2.0**-24)
    for U in (U1.cpu().numpy(), U2.cpu().numpy()):
        assert (np.abs(U - U_ref) <= tol * aU + 1e-30).all(), np.abs(U - U_ref).max()
