"""Measured comparison of the two adjoint designs (Sec. III-B: U = P^T dL/dR
with the straight-through estimator) on one workload:

* the variable-major gather of the update kernels (tsat_bwd_dev: the
  forward's planes of R gathered per variable by record windows, U written
  once, no atomics), and
* the clause-major scatter (tsat_bwd_scatter_dev: one thread per clause and
  32 candidates adds dL/dR[R] into every literal's row of U with FP32
  atomics, the first literal of each clause through an LDS tile).

Both calls include the forward pass and SmoothMin that produce dL/dR.

    python -m paper_2511_07737_amd.adjoint_ab [--workload large|structured] [--reps 5]

prints one JSON line: ms per call of each design, the largest difference
between their U and the largest |U|.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2511_07737_amd import gen, tsat  # noqa: E402


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", choices=["large", "structured"], default="large")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    import torch

    if args.workload == "large":
        cnf, N = gen.planted_ksat(1_000_000, 4_100_000, 3, seed=1), 256
    else:
        cnf, N = gen.structured(500_000, 2_500_000, seed=2), 128
    print(f"[adjoint_ab] {args.workload}: V={cnf.num_vars} C={cnf.num_clauses} N={N}", file=sys.stderr, flush=True)
    s = tsat.Solver()
    s.load(cnf)
    b = (np.random.default_rng(1).random((cnf.num_vars, N)) < 0.5).astype(np.uint8)
    bits = torch.tensor(tsat.pack_bits(b).view(np.int64), device="cuda")
    dS = torch.full((N,), -1.0, dtype=torch.float32, device="cuda")  # the loss -sum S
    U = {k: torch.empty((cnf.num_vars, N), dtype=torch.float32, device="cuda") for k in ("gather", "scatter")}
    calls = {"gather": s.bwd_dev, "scatter": s.bwd_scatter_dev}
    st = torch.cuda.current_stream().cuda_stream
    out = {"workload": args.workload, "V": cnf.num_vars, "C": cnf.num_clauses, "L": cnf.num_lits, "N": N}
    for name, f in calls.items():
        f(bits.data_ptr(), N, 1.0, dS.data_ptr(), U[name].data_ptr(), st)  # untimed first call
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.reps):
            f(bits.data_ptr(), N, 1.0, dS.data_ptr(), U[name].data_ptr(), st)
        torch.cuda.synchronize()
        out[f"{name}_ms"] = (time.perf_counter() - t0) / args.reps * 1e3
        print(f"[adjoint_ab] {name}: {out[f'{name}_ms']:.3f} ms per call", file=sys.stderr, flush=True)
    out["max_abs_diff"] = (U["gather"] - U["scatter"]).abs().max().item()
    out["max_abs_U"] = U["gather"].abs().max().item()
    out["atomics_per_call"] = cnf.num_lits * N
    s.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
