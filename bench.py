#!/usr/bin/env python3
"""Benchmark of the gfx950 gradient-guided SAT step (TurboSAT, arXiv 2511.07737).

One step = one pass of the whole hot path over the batch: forward histogram
of R = P A (all width buckets) -> SmoothMin/loss/dL/dR table -> fused
variable-major adjoint + Eq. 5 backward + AdamW + re-binarization.

Default workload: planted random 3-SAT, V = 1,000,000, C = 4,100,000
(ratio 4.1), N = 256 candidates, FP32 logits and optimizer state, inputs
resident in HBM before the timed region.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps 2000] [--warmup 10]
                       [--workload large|structured|tiny] [--no-cpu-baseline]
                       [--no-learned] [--no-ragged] [--no-structured] [--no-stream]
                       [--no-autotune] [--calib-copy-mib M]

Besides the timed workload the line carries the bandwidth reference kernels,
the tiny-configuration steps-to-SAT distribution, the learned-versus-random
start comparison, the structured configuration, the ragged 1000-instance
configuration and the FP64 oracle timed on the host (one thread and all
threads).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

WORKLOADS = {
    "large": dict(kind="planted", V=1_000_000, C=4_100_000, N=256, seed=1, init_seed=1001,
                  name="planted random 3-SAT, V=1e6, C=4.1e6 (ratio 4.1), N=256 restarts, FP32 logits"),
    "structured": dict(kind="structured", V=500_000, C=2_500_000, N=128, seed=2, init_seed=1002,
                       name="structured planted CNF, V=5e5, C=2.5e6, widths 2-12 P(k)~k^-2.5, "
                            "power-law occurrences (2.2) in 64 communities, N=128"),
    "tiny": dict(kind="planted", V=200, C=800, N=64, seed=1, init_seed=1001,
                 name="planted random 3-SAT, V=200, C=800, N=64"),
}


def make_cnf(w):
    from paper_2511_07737_amd import gen

    if w["kind"] == "planted":
        return gen.planted_ksat(w["V"], w["C"], 3, seed=w["seed"])
    return gen.structured(w["V"], w["C"], seed=w["seed"])


def uses_clause_planes(cnf, N, planes_on):
    """The update gathers the forward's planes of R: every clause at most 15
    wide and at most 256 candidates."""
    import numpy as np

    w = cnf.widths()
    return bool(planes_on) and w.size > 0 and int(w.max()) <= 15 and N <= 256


def model_bytes(cnf, N):
    """Algorithmic bytes of the path's byte model (per iteration):
    - update: clause indices (4 B per literal), the current value rows
      (V N / 8), theta, m, v read and written (24 B per (variable,
      candidate)) and the next value rows (V N / 8);
    - fwd: clause codes (4 B per literal) and every value row once (V N / 8);
    - fwdbwd: the forward and the adjoint as separate passes, codes read
      twice, rows read twice, the FP32 gradient written once: 8 L + V N / 4 + 4 V N;
    - step_fused_min: fwd + update (the fused design never moves U);
    - step_unfused: fwdbwd plus an update that reads U: + 28.125 V N."""
    V, L = cnf.num_vars, cnf.num_lits
    VN = V * N
    upd = 4 * L + VN / 8 + 24 * VN + VN / 8
    fwd = 4 * L + VN / 8
    fwdbwd = 8 * L + VN / 4 + 4 * VN
    return dict(update=upd, fwd=fwd, fwdbwd=fwdbwd, step_fused_min=fwd + upd, step_unfused=fwdbwd + 28.125 * VN)


def implementation_bytes(cnf, N, planes):
    """What the kernels of this implementation move at least once per
    iteration beyond the byte model (reported separately): with clause
    planes, the forward writes and the update reads R of every clause in
    binary (P planes of J words, P = 2 up to width 3, else 4, J = row words);
    row means (16 B per variable) and record offsets (8 B per variable); the
    update writes both literal rows (the complement too)."""
    import numpy as np

    V, C = cnf.num_vars, cnf.num_clauses
    W = (N + 63) // 64
    J = W if W <= 2 else (4 if W <= 4 else 8 * ((W + 7) // 8))
    out = dict(means_offsets=24 * V, complement_rows=V * W * 8)
    if planes:
        # two planes per clause of width <= 3, four per wider clause
        w = cnf.widths()
        rows = 2 * int((w <= 3).sum()) + 4 * int((w > 3).sum())
        out["planes_write"] = out["planes_read"] = int(rows * J * 8)
    else:
        occ_words = int((cnf.widths().astype(np.int64) ** 2).sum())
        out["occurrence_records"] = 4 * occ_words
    return out


def frac_entry(nbytes, ms, kernel=None):
    gbs = nbytes / (ms * 1e-3) / 1e9
    e = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": int(nbytes), "ms": round(ms, 5)}
    if kernel:
        e["kernel"] = kernel
    return e


KERNEL_SOURCES = ["paper_2511_07737_amd/csrc/tsat_kernels.hip", "paper_2511_07737_amd/csrc/tsat_device.h"]
PROFILE_FILES = {"large": "profiles/var_window_kernel__planted-3sat_V1e6_C4.1e6_N256.txt",
                 "structured": "profiles/var_window_levels_kernel__structured_V5e5_C2.5e6_N128.txt"}


def measured_traffic(workload):
    """Bytes per launch of the dominant kernel between L2 and the memory
    fabric, from the committed rocprofv3 counter summary (read and write
    requests times their sizes, the sizes read off a copy kernel of known
    bytes), or None when there is none or the kernel sources changed since."""
    import hashlib

    path = PROFILE_FILES.get(workload)
    if not path or not os.path.exists(os.path.join(ROOT, path)):
        return None
    fields = {}
    for line in open(os.path.join(ROOT, path)):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def learned_vs_random():
    """The learned proposal's start against the majority-vote start
    (Laplace-smoothed positive-occurrence fraction) and the N(0,1) start:
    on 20 held-out planted 3-SAT instances V = 100,000, C = 410,000 (seeds
    20000..20019), 128 restarts, one batch per arm (steps to the 99%
    hand-off, lowest unsatisfied count vs step, censored steps and time to
    all-SAT); and steps to all-SAT per instance on 400 small held-out
    instances, where the search reaches all-SAT."""
    from paper_2511_07737_amd import learned

    if not os.path.exists(learned.DEFAULT_WEIGHTS):
        return None
    print("[bench] learned vs random start", file=sys.stderr, flush=True)
    weights, meta = learned.load_weights()
    res = learned.evaluate_heldout(weights, count=20, V=100_000, restarts=128, max_steps=3600)
    print("[bench] learned vs random start: small-instance batch", file=sys.stderr, flush=True)
    res["small_batch"] = learned.compare_batch(weights, count=400, vmin=200, vmax=1000, ratio=4.0)
    res["training"] = {k: meta.get(k) for k in ("instances", "rows", "val_accuracy", "final_loss", "epochs")}
    return res


def mixing_block():
    """Assignment mixing at the learning-rate restarts (every 360 iterations)
    against the plain schedule, none-mode tau = 2: the tiny configuration
    (32 instances, 1500 iterations, freeze on SAT: solved count and steps to
    SAT) and the large one (2000 iterations: steps to the 99% hand-off and
    the best candidate's unsatisfied clauses at the end and at each
    restart)."""
    import numpy as np

    from paper_2511_07737_amd import gen, tsat

    print("[bench] mixing at restarts", file=sys.stderr, flush=True)
    out = {}
    cnfs = [gen.planted_ksat(200, 800, 3, seed=j) for j in range(1, 33)]
    th = np.concatenate([gen.normal_logits(200, 64, 1000 + j) for j in range(1, 33)])
    tiny = {"workload": "32 planted 3-SAT instances V=200, C=800, N=64, 1500 iterations, none-mode tau=2"}
    for mix in (0, 1):
        s = tsat.Solver(params=tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0, mix=mix))
        s.load_batch(cnfs)
        s.init_batch(64, init_logits=th)
        s.set_graph(True)
        s.step(1500, stop_on_sat=True)
        sat = np.array([x["first_sat_step"] for x in s.instance_status()])
        s.close()
        q = [float(v) for v in np.percentile(sat[sat >= 0], [10, 50, 90])] if (sat >= 0).any() else None
        tiny["mix" if mix else "plain"] = {"solved": int((sat >= 0).sum()), "steps_to_sat_p10_p50_p90": q,
                                            "solved_after_360": int((sat >= 360).sum())}
    out["tiny"] = tiny
    cnf = gen.planted_ksat(1_000_000, 4_100_000, 3, seed=1)
    th = gen.normal_logits(cnf.num_vars, 256, 1001)
    large = {"workload": "planted 3-SAT V=1e6, C=4.1e6, N=256, 2000 iterations, none-mode tau=2"}
    for mix in (0, 1):
        s = tsat.Solver(params=tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0, mix=mix))
        s.load(cnf)
        s.init_batch(256, init_logits=th)
        best = []
        done, first99 = 0, -1
        for stop in (360, 720, 1080, 1440, 1800, 2000):
            r = s.step(stop - done)
            done = stop
            first99 = r.first_converged_step
            best.append(int(cnf.num_clauses - r.best_sat_count))
        s.close()
        large["mix" if mix else "plain"] = {"steps_to_99": first99, "best_unsat_at_360_720_1080_1440_1800_2000": best}
    out["large"] = large
    return out


def ragged_block(count, max_steps):
    """The ragged many-instance configuration: `count` planted 3-SAT
    instances (V log-uniform in [1e3, 2e5], ratio uniform in [3.8, 4.2],
    seeds 3000 + j), 32 restarts each, one batch replayed from a captured
    graph with autotuned launch shapes; hand-off phase (stop mode 2), then
    from the same start to all-SAT or the step cap (censored percentiles)."""
    from paper_2511_07737_amd import ragged, tsat

    print(f"[bench] ragged: generating {count} instances", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    cnfs = ragged.generate(count, workers=min(16, os.cpu_count() or 1))
    t_gen = time.perf_counter() - t0
    params = tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)
    out = ragged.solve_batch(cnfs, 32, max_steps, params, autotune_iters=2, graph=True)
    L = out["total_lits"]
    out["gen_s"] = round(t_gen, 1)
    out["workload"] = (f"{count} planted 3-SAT instances, V log-uniform in [1000, 200000], ratio uniform in "
                       f"[3.8, 4.2], 32 restarts each, none-mode tau=2, cap {max_steps} steps")
    # throughput of the batch iteration (hand-off phase, every instance live)
    ms = out["handoff"]["ms_per_step"]
    out["evals_per_s"] = L * 32 / (ms * 1e-3)
    V = out["total_vars"]
    step_min = 4 * L + V * 32 / 8 + 4 * L + V * 32 / 8 + 24 * V * 32 + V * 32 / 8
    out["step_frac_fused_min"] = round(step_min / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def structured_block(steps):
    """The structured configuration (community-structured planted CNF,
    V = 5e5, C = 2.5e6, widths 2-12, N = 128) as a report of the default
    run: the same measurement as --workload structured, autotuned, 10
    warmup and `steps` timed iterations."""
    import numpy as np

    from paper_2511_07737_amd import gen, tsat

    w = WORKLOADS["structured"]
    print("[bench] structured: generating", file=sys.stderr, flush=True)
    cnf = make_cnf(w)
    N = w["N"]
    s = tsat.Solver(device=0)
    s.load(cnf)
    s.init_batch(N, init_logits=gen.normal_logits(cnf.num_vars, N, w["init_seed"]))
    cfg, used = s.autotune(iters=2)
    s.step(10)
    s.set_timing(True)
    t0 = time.perf_counter()
    s.step(steps)
    t1 = time.perf_counter()
    s.set_timing(False)
    kms, _ = s.get_timing()
    launch = s.launch_config().as_dict()
    s.close()
    ms = 1e3 * (t1 - t0) / steps
    sb = model_bytes(cnf, N)
    upd = frac_entry(sb["update"], kms[2], "var_step")
    upd["traffic"] = measured_traffic("structured")
    return {"workload": w["name"], "V": cnf.num_vars, "C": cnf.num_clauses, "L": cnf.num_lits, "N": N,
            "steps": steps, "ms_per_step": round(ms, 5), "evals_per_s": cnf.num_lits * N / (ms * 1e-3),
            "kernels_ms": {n: round(x, 5) for n, x in zip(["fwd_hist", "smin_tables", "var_step"], kms)},
            "roofline": upd, "roofline_fwd": frac_entry(sb["fwd"], kms[0], "fwd_hist"),
            "frac_fused_min": round(sb["step_fused_min"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launch": launch, "autotune_iterations": used}


def tiny_distribution():
    """Steps to all-SAT and to the 99% hand-off on the tiny configuration:
    32 planted 3-SAT instances V = 200, C = 800 (seeds 1..32), N = 64 with
    N(0,1) starts (seeds 1001..1032), 500 iterations, solved as one batch
    that freezes each instance on its first satisfying candidate; for the
    method's default setting (Eq. 5 mean normalization, tau = 1) and for the
    none-mode setting the learned proposal uses (tau = 2)."""
    import numpy as np

    from paper_2511_07737_amd import gen, tsat

    cnfs = [gen.planted_ksat(200, 800, 3, seed=j) for j in range(1, 33)]
    th = np.concatenate([gen.normal_logits(200, 64, 1000 + j) for j in range(1, 33)])
    out = {"workload": "32 planted 3-SAT instances V=200, C=800, N=64, 500 iterations"}
    for name, p in (("mean_tau1", tsat.default_params()),
                    ("none_tau2", tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0))):
        s = tsat.Solver(params=p)
        s.load_batch(cnfs)
        s.init_batch(64, init_logits=th)
        s.set_graph(True)
        t0 = time.perf_counter()
        rep = s.step(500, stop_on_sat=True)
        wall = time.perf_counter() - t0
        st = s.instance_status()
        s.close()
        sat = np.array([x["first_sat_step"] for x in st])
        conv = np.array([x["first_converged_step"] for x in st])
        q = lambda x: [float(v) for v in np.percentile(x, [10, 50, 90])] if x.size else None  # noqa: E731
        out[name] = {"solved": int((sat >= 0).sum()), "steps_to_sat_p10_p50_p90": q(sat[sat >= 0]),
                     "reached_99": int((conv >= 0).sum()), "steps_to_99_p10_p50_p90": q(conv[conv >= 0]),
                     "iterations_run": rep.steps_done, "steps_per_s": rep.steps_done / wall}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_step_threaded(oc, th, m, v, t, threads):
    """One oracle iteration (Eq. 5 + Eq. 2, R histogram, SmoothMin, adjoint,
    Eq. 5 backward, AdamW) with each stage's oracle routine run on
    `threads` parts at once: variables for the row-wise stages, candidates
    for the histogram and the adjoint (each part on a copy of its columns)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle as orc

    V, N = th.shape
    p = orc.default_params()
    rows = np.array_split(np.arange(V), threads)
    cols = np.array_split(np.arange(N), threads)
    b = np.empty((V, N), dtype=np.uint8)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        def binarize(r):
            if r.size:
                b[r[0]:r[-1] + 1], _ = orc.binarize(th[r[0]:r[-1] + 1], p.mode)
        list(ex.map(binarize, rows))
        H = np.zeros((N, oc.K + 1), dtype=np.int64)

        def hist(c):
            if c.size:
                H[c[0]:c[-1] + 1] = orc.histogram(oc, np.ascontiguousarray(b[:, c[0]:c[-1] + 1]))
        list(ex.map(hist, cols))
        _, table, _ = orc.smoothmin(H, p.tau)
        U = np.empty((V, N))

        def adj(c):
            if c.size:
                U[:, c[0]:c[-1] + 1] = orc.adjoint(oc, np.ascontiguousarray(b[:, c[0]:c[-1] + 1]),
                                                   np.ascontiguousarray(table[c[0]:c[-1] + 1]))
        list(ex.map(adj, cols))
        g = np.empty((V, N))

        def nb(r):
            if r.size:
                g[r[0]:r[-1] + 1] = orc.norm_backward(th[r[0]:r[-1] + 1], U[r[0]:r[-1] + 1], p.mode)
        list(ex.map(nb, rows))
        lr = orc.lr(t, p)

        def adam(r):
            if r.size:
                sl = slice(r[0], r[-1] + 1)
                orc.adamw(th[sl], m[sl], v[sl], g[sl], lr, t + 1)
        list(ex.map(adam, rows))


def cpu_baseline(cnf, w, n_sample, threads, steps_all):
    """The FP64 oracle on the host: one single-threaded iteration on
    n_sample of the candidates (orc.step), and `steps_all` iterations over
    all candidates with every stage split over `threads` threads."""
    import numpy as np

    import oracle as orc
    from paper_2511_07737_amd import gen

    oc = orc.Cnf.from_gen(cnf)
    N = w["N"]
    th = gen.normal_logits(cnf.num_vars, n_sample, w["init_seed"]).astype(np.float64)
    t0 = time.perf_counter()
    orc.step(oc, th, np.zeros_like(th), np.zeros_like(th), 0)
    dt1 = time.perf_counter() - t0
    single = dict(value=cnf.num_lits * n_sample / dt1, cores=1, seconds=round(dt1, 2),
                  sample=f"one oracle iteration (orc.step) with {n_sample} of the {N} candidates")
    th = gen.normal_logits(cnf.num_vars, N, w["init_seed"]).astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    t0 = time.perf_counter()
    for t in range(steps_all):
        oracle_step_threaded(oc, th, m, v, t, threads)
    dt = time.perf_counter() - t0
    return dict(value=cnf.num_lits * N * steps_all / dt, unit="clause-literal evals/s", cores=threads, kind="oracle",
                sample=f"{steps_all} oracle iterations over the whole instance and all {N} candidates, every stage "
                       f"(binarize, R histogram, SmoothMin, adjoint, Eq. 5 backward, AdamW) split over {threads} "
                       f"threads; {dt:.1f} s C FP64",
                cpu_model=cpu_model(), single_thread=single, seconds=dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=128, help="candidates of the single-threaded oracle iteration")
    ap.add_argument("--cpu-steps", type=int, default=3, help="all-candidate oracle iterations on all host threads")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the solve-quality reports: the learned-versus-random start comparison and the "
                         "tiny-configuration steps-to-SAT distribution")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged many-instance configuration")
    ap.add_argument("--no-structured", action="store_true",
                    help="skip the structured-configuration report of a run on another workload")
    ap.add_argument("--structured-steps", type=int, default=500)
    ap.add_argument("--ragged-count", type=int, default=1000)
    ap.add_argument("--ragged-steps", type=int, default=3600)
    ap.add_argument("--no-stream", action="store_true", help="skip the bandwidth reference kernels")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, launch one plain device copy kernel of this many MiB (read + write), "
                         "the reference point for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding over candidates is "
                                   "a design note, not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np

    from paper_2511_07737_amd import gen, tsat

    w = WORKLOADS[args.workload]
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    cnf = make_cnf(w)
    N = w["N"]
    s = tsat.Solver(device=0)
    s.load(cnf)
    s.init_batch(N, init_logits=gen.normal_logits(cnf.num_vars, N, w["init_seed"]))
    print("[bench] warmup", file=sys.stderr, flush=True)
    tuned = None
    if args.warmup > 0 and not args.no_autotune:
        # launch shapes never change results: tuning iterations are ordinary
        # (untimed) iterations of the run
        cfg, used = s.autotune(iters=2)
        tuned = dict(cfg.as_dict(), iterations=used)
    s.step(args.warmup)
    s.set_timing(True)
    t0 = time.perf_counter()
    rep = s.step(args.steps)  # synchronous: returns after the last kernel completes
    t1 = time.perf_counter()
    s.set_timing(False)
    kms, kiters = s.get_timing()
    sec = t1 - t0
    evals_per_step = cnf.num_lits * N
    ms_per_step = 1e3 * sec / args.steps
    value = evals_per_step * args.steps / sec

    planes = uses_clause_planes(cnf, N, s.launch_config().clause_planes)
    sb = model_bytes(cnf, N)
    impl = implementation_bytes(cnf, N, planes)
    names = ["fwd_hist", "smin_tables", "var_step"]
    dom = int(np.argmax(kms))
    roofline = None
    if dom in (0, 2):
        roofline = frac_entry(sb["update"] if dom == 2 else sb["fwd"], kms[dom], names[dom])
        roofline["traffic"] = measured_traffic(args.workload) if dom == 2 else None
        roofline["impl_bytes_per_launch"] = {k: v for k, v in impl.items()
                                             if dom == 2 or k == "planes_write"}
    out = {
        "metric": "clause-literal evals/s (fwd+bwd, % HBM peak); steps-to-all-SAT learned vs random",
        "value": value,
        "unit": "clause-literal evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "V": cnf.num_vars, "C": cnf.num_clauses, "L": cnf.num_lits, "N": N,
                   "steps_per_launch_sequence": args.steps, "launch": s.launch_config().as_dict(),
                   "autotuned": tuned is not None},
        "roofline": roofline,
        # the forward (and exact clause check) against its own byte model
        "roofline_fwd": frac_entry(sb["fwd"], kms[0], "fwd_hist"),
        # the whole iteration against the fused minimum (forward + update:
        # U never reaches memory) and against the unfused byte model
        "roofline_step": {"ms_per_step": round(ms_per_step, 5),
                          "bytes_fused_min": int(sb["step_fused_min"]),
                          "frac_fused_min": round(sb["step_fused_min"] / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "bytes_unfused": int(sb["step_unfused"]),
                          "frac_unfused": round(sb["step_unfused"] / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        # the metric's fwd+bwd byte model over the smallest timed region that
        # holds forward and backward (the whole iteration: the backward is
        # fused with the update)
        "roofline_fwdbwd": {"bytes": int(sb["fwdbwd"]), "ms": round(ms_per_step, 5),
                            "frac": round(sb["fwdbwd"] / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "evals_per_s": value},
        "kernels_ms": {n: round(x, 5) for n, x in zip(names, kms)},
        "kernel_iters": kiters,
        "best_sat_count": rep.best_sat_count,
        "first_sat_step": rep.first_sat_step,
        # the exact clause check is the forward histogram: bin 0 counts the
        # unsatisfied clauses of every candidate
        "check_pairs_per_s": cnf.num_clauses * N / (kms[0] * 1e-3),
    }
    if not args.no_stream:
        # bandwidth references on 1 GiB arrays: the practical ceilings the
        # fractions above can be read against
        nb = 1 << 30
        ref = {}
        for kind, name, moved in ((0, "copy_x4", 2), (1, "rw3_x4", 6), (2, "rw3_rows", 6)):
            ms = s.stream_calibrate(nb, kind, reps=5)
            ref[name] = {"gbs": round(moved * nb / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4)}
        out["stream_ceiling"] = ref
    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        ms = s.copy_calibrate(nb)  # one copy kernel: nb bytes read, nb bytes written
        out["calib_copy"] = {"bytes": nb, "ms": ms, "gbs": round(2 * nb / (ms * 1e-3) / 1e9, 1)}
    s.close()
    if not args.no_learned:
        out["tiny"] = tiny_distribution()
        out["learned_vs_random"] = learned_vs_random()
        out["mixing"] = mixing_block()
    if not args.no_structured and args.workload != "structured":
        out["structured"] = structured_block(args.structured_steps)
    if not args.no_ragged:
        out["ragged"] = ragged_block(args.ragged_count, args.ragged_steps)
    if not args.no_cpu_baseline:
        threads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))
        print(f"[bench] cpu baseline (oracle, 1 and {threads} threads)", file=sys.stderr, flush=True)
        cb = cpu_baseline(cnf, w, min(args.cpu_sample, N), threads, args.cpu_steps)
        out["cpu_baseline"] = {k: v for k, v in cb.items() if k != "seconds"}
        out["gpu_over_cpu"] = value / cb["value"]
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
