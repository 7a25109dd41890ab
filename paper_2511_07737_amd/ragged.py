"""Batched ragged solve: many planted 3-SAT instances of uneven size solved as
one batch on one GPU.

The instances form one block-diagonal CNF; every instance keeps its own
Eq. 5 row means (over its own candidates), histogram, SmoothMin table and
schedule state, and freezes once one of its candidates satisfies every clause
(the exact check of Sec. III-A).  The iterations are replayed from a captured
HIP graph and the host only polls the stop flag; per-instance device
timestamps give the time to the first satisfying candidate.  Launch shapes
come from the library's autotuner.

    python -m paper_2511_07737_amd.ragged [--count 1000] [--restarts 32]
        [--max-steps 3600] [--mode none] [--tau 2] [--autotune-iters 2]

prints one JSON line with instances/s to the hand-off point and to SAT, the
solved fraction and the p50/p99 time- and steps-to-hand-off and -to-SAT over
all instances (unsolved instances are censored at the step cap: a percentile
past the solved fraction is null).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2511_07737_amd import gen, tsat  # noqa: E402


def _make(args):
    j, seed, vmin, vmax, rlo, rhi = args
    return gen.ragged_instance(j, seed, vmin, vmax, rlo, rhi)


def generate(count: int, seed: int = 3000, vmin: int = 1000, vmax: int = 200000, ratio_lo: float = 3.8,
             ratio_hi: float = 4.2, workers: int = 8) -> list:
    """gen.ragged_set drawn over a process pool (same instances, same order)."""
    jobs = [(j, seed, vmin, vmax, ratio_lo, ratio_hi) for j in range(count)]
    if workers <= 1 or count < 16:
        return [_make(a) for a in jobs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_make, jobs, chunksize=8))


def censored_percentile(values, n_total: int, q: float):
    """q-th percentile over n_total instances of which only len(values) have
    an observed value; the others are censored (beyond the step cap, larger
    than every observed value).  Order statistic of rank ceil(q/100 n_total):
    None when that rank falls among the censored instances."""
    if n_total <= 0:
        return None
    k = max(1, int(np.ceil(q / 100.0 * n_total)))
    xs = np.sort(np.asarray(values, dtype=np.float64))
    return float(xs[k - 1]) if k <= xs.size else None


def witness_holds(cnf, vals: np.ndarray, device: int = 0) -> bool:
    """The library's exact clause check (Sec. III-A) of one instance's
    witness, in a solver of its own."""
    s = tsat.Solver(device=device)
    try:
        s.load(cnf)
        _, is_sat = s.check_bits(tsat.pack_bits(vals.reshape(-1, 1).astype(np.uint8)), 1)
        return bool(is_sat[0])
    finally:
        s.close()


def log(msg: str) -> None:
    print(f"[ragged] {msg}", file=sys.stderr, flush=True)


def run_steps(s, max_steps: int, stop_mode: int, chunk: int = 200):
    """tsat_step in chunks (the stop state carries over between calls),
    reporting progress; returns the total steps done and the last report."""
    done, rep = 0, None
    while done < max_steps:
        rep = s.step(min(chunk, max_steps - done), stop_on_sat=stop_mode)
        done += rep.steps_done
        st = s.instance_status()
        frozen = sum(x["frozen"] for x in st)
        log(f"step {done}: {frozen}/{len(st)} instances frozen")
        if frozen == len(st) or rep.steps_done == 0:
            break
    return done, rep


def solve_batch(cnfs, restarts: int, max_steps: int, params, seed: int = 1, autotune_iters: int = 2,
                graph: bool = True, verify: bool = True, device: int = 0) -> dict:
    s = tsat.Solver(device=device, params=params)
    t0 = time.perf_counter()
    s.load_batch(cnfs)
    t_load = time.perf_counter() - t0
    log(f"loaded in {t_load:.1f} s")
    tune = None
    if autotune_iters > 0:
        s.init_batch(restarts, seed=seed)
        c, used = s.autotune(autotune_iters)
        tune = dict(c.as_dict(), iterations=used)
        log(f"autotuned: {tune}")
    hz = s.device_clock_hz()
    n = len(cnfs)
    out = {
        "instances": n,
        "restarts": restarts,
        "total_vars": int(sum(c.num_vars for c in cnfs)),
        "total_clauses": int(sum(c.num_clauses for c in cnfs)),
        "total_lits": int(sum(c.num_lits for c in cnfs)),
        "load_s": t_load,
        "launch_config": tune,
    }
    # phase 1: until every instance hands off (converged or satisfied)
    s.init_batch(restarts, seed=seed)  # the timed solve starts fresh
    s.set_graph(graph)
    t0 = time.perf_counter()
    steps1, rep = run_steps(s, max_steps, 2)
    wall = time.perf_counter() - t0
    st = s.instance_status()
    done = [j for j, x in enumerate(st) if x["frozen"]]
    tth = [((x["sat_ticks"] if x["first_sat_step"] >= 0 and (x["first_converged_step"] < 0 or
             x["first_sat_step"] <= x["first_converged_step"]) else x["conv_ticks"]) - x["start_ticks"]) / hz
           for x in (st[j] for j in done)]
    hsteps = [min(x for x in (st[j]["first_sat_step"], st[j]["first_converged_step"]) if x >= 0) for j in done]
    out["handoff"] = {
        "handed_off": len(done), "frac": len(done) / n, "steps_done": steps1, "wall_s": wall,
        "ms_per_step": 1e3 * wall / max(1, steps1),
        "instances_per_s_handed_off": len(done) / wall if wall > 0 else None,
        # over all n instances; an instance not handed off within the cap is censored
        "p50_time_s": censored_percentile(tth, n, 50), "p99_time_s": censored_percentile(tth, n, 99),
        "p50_steps": censored_percentile(hsteps, n, 50), "p99_steps": censored_percentile(hsteps, n, 99),
    }
    # phase 2: from the same start until every instance is satisfied or the cap
    s.init_batch(restarts, seed=seed)
    t0 = time.perf_counter()
    steps2, rep = run_steps(s, max_steps, 1)
    wall = time.perf_counter() - t0
    st = s.instance_status()
    solved = [j for j, x in enumerate(st) if x["first_sat_step"] >= 0]
    tts = [(st[j]["sat_ticks"] - st[j]["start_ticks"]) / hz for j in solved]
    steps = [st[j]["first_sat_step"] for j in solved]
    bad = []
    if verify:
        for j in solved:
            vals, _ = s.get_witness_instance(j, cnfs[j].num_vars)
            if not witness_holds(cnfs[j], vals, device):
                bad.append(j)
    conv = [j for j, x in enumerate(st) if x["first_converged_step"] >= 0]
    s.close()
    out.update({
        "solved": len(solved),
        "solved_frac": len(solved) / n,
        "converged_frac": len(conv) / n,
        "witnesses_failing_host_check": len(bad),
        "steps_done": steps2,
        "wall_s": wall,
        "ms_per_step": 1e3 * wall / max(1, steps2),
        "instances_per_s_solved": len(solved) / wall if wall > 0 else None,
        # percentiles over all n instances: unsolved ones are censored at the
        # step cap, so a percentile beyond the solved fraction is None
        "censored": len(solved) < n,
        "p50_time_to_sat_s": censored_percentile(tts, n, 50),
        "p99_time_to_sat_s": censored_percentile(tts, n, 99),
        "p50_steps_to_sat": censored_percentile(steps, n, 50),
        "p99_steps_to_sat": censored_percentile(steps, n, 99),
    })
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--count", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--vmin", type=int, default=1000)
    ap.add_argument("--vmax", type=int, default=200000)
    ap.add_argument("--restarts", type=int, default=32)
    ap.add_argument("--max-steps", type=int, default=3600)
    ap.add_argument("--mode", choices=["none", "mean"], default="none")
    ap.add_argument("--tau", type=float, default=2.0)
    ap.add_argument("--autotune-iters", type=int, default=2)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    print(f"[ragged] generating {args.count} instances", file=sys.stderr, flush=True)
    cnfs = generate(args.count, args.seed, args.vmin, args.vmax, workers=args.workers)
    t_gen = time.perf_counter() - t0
    print(f"[ragged] generated in {t_gen:.1f} s; solving", file=sys.stderr, flush=True)
    params = tsat.default_params(norm_mode=tsat.MODE_NONE if args.mode == "none" else tsat.MODE_MEAN, tau=args.tau)
    out = solve_batch(cnfs, args.restarts, args.max_steps, params, autotune_iters=args.autotune_iters,
                      graph=not args.no_graph)
    out.update(metric="ragged batch: instances/s, p50/p99 time-to-SAT", mode=args.mode, tau=args.tau,
               workload=f"{args.count} planted 3-SAT instances, V log-uniform in [{args.vmin}, {args.vmax}], "
                        f"ratio uniform in [3.8, 4.2], {args.restarts} restarts each", gen_s=t_gen)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
