"""Learned proposal: a corpus of planted 3-SAT instances labelled by the solver
itself, training of the per-variable network on the GPU with the library's
forward / backward / Adam kernels, and the learned-versus-random comparison
of steps- and time-to-all-SAT on a held-out instance.

The network (16 features -> 128 -> 128 -> 1, BF16 weights, FP32 accumulation
on MFMA) proposes P(x_v = true); the batch then starts from draws of that
proposal (tsat_init_from_proposal) instead of N(0,1) logits.  Labels are the
assignments the gradient search converges to: per instance, its satisfying
candidate if one was found, else its best candidate once more than 99% of
the clauses were satisfied; instances that never converge give no labels.

    python -m paper_2511_07737_amd.learned train [--instances 5000] [--out W.npz]
    python -m paper_2511_07737_amd.learned compare --weights W.npz
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

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "proposal_mlp.npz")

# FP32 parameter vector layout (include/tsat.h): W1 [16][128], b1, W2 [128][128], b2, w3, b3
SHAPES = (("W1", (16, 128)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("w3", (128,)), ("b3", (1,)))


def log(msg: str) -> None:
    print(f"[learned] {msg}", file=sys.stderr, flush=True)


def init_params(seed: int) -> np.ndarray:
    """He-style initial parameters as the flat FP32 vector."""
    g = np.random.default_rng(seed)
    parts = {
        "W1": g.normal(0, np.sqrt(2.0 / 16), (16, 128)), "b1": np.zeros(128),
        "W2": g.normal(0, np.sqrt(2.0 / 128), (128, 128)), "b2": np.zeros(128),
        "w3": g.normal(0, np.sqrt(1.0 / 128), 128), "b3": np.zeros(1),
    }
    return np.concatenate([np.asarray(parts[k], np.float64).ravel() for k, _ in SHAPES]).astype(np.float32)


# --------------------------------------------------------------------------
# corpus and self-labelling
# --------------------------------------------------------------------------

def _corpus_instance(args):
    j, seed, vmin, vmax, ratio = args
    g = gen.rng(seed + j)
    V = int(g.integers(vmin, vmax + 1))
    return gen.planted_ksat(V, int(round(ratio * V)), 3, seed=(seed + j) * 7919 + 3)


def corpus(count: int, seed: int = 50_000, vmin: int = 20_000, vmax: int = 100_000, ratio: float = 4.1,
           workers: int = 8):
    """Planted 3-SAT instances, V uniform in [vmin, vmax], C = ratio * V."""
    from concurrent.futures import ProcessPoolExecutor

    jobs = [(j, seed, vmin, vmax, ratio) for j in range(count)]
    if workers <= 1:
        return [_corpus_instance(a) for a in jobs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_corpus_instance, jobs, chunksize=4))


def column_bits(packed_rows: np.ndarray, cand: int) -> np.ndarray:
    """0/1 values of candidate `cand` from bit-packed rows [V][W]."""
    return ((packed_rows[:, cand // 64] >> np.uint64(cand % 64)) & np.uint64(1)).astype(np.uint8)


def label_chunk(cnfs, restarts: int, max_steps: int, params, seed: int, rows_per_instance: int, rng,
                device: int = 0):
    """Solve one batch of instances and return (features, labels, stats) of
    the converged instances (at most rows_per_instance random rows each)."""
    s = tsat.Solver(device=device, params=params)
    s.load_batch(cnfs)
    s.init_batch(restarts, seed=seed)
    s.set_graph(True)
    s.step(max_steps, stop_on_sat=2)  # every instance stops at its hand-off point
    st = s.instance_status()
    bits = s.get_bits()
    X = s.get_features()
    s.close()
    xs, ys = [], []
    n_sat = n_conv = 0
    base = 0
    for j, c in enumerate(cnfs):
        info = st[j]
        rows = slice(base, base + c.num_vars)
        base += c.num_vars
        if info["first_sat_step"] >= 0:
            cand = info["sat_candidate"]
            n_sat += 1
        elif info["first_converged_step"] >= 0:
            cand = info["best_candidate"]
        else:
            continue
        n_conv += 1
        y = column_bits(bits[rows], cand)
        pick = np.arange(c.num_vars)
        if rows_per_instance and c.num_vars > rows_per_instance:
            pick = np.sort(rng.choice(c.num_vars, rows_per_instance, replace=False))
        xs.append(X[rows][pick])
        ys.append(y[pick])
    if not xs:
        return np.zeros((0, 16), np.float32), np.zeros(0, np.float32), dict(sat=0, converged=0)
    return np.concatenate(xs), np.concatenate(ys).astype(np.float32), dict(sat=n_sat, converged=n_conv)


def build_dataset(cnfs, restarts=32, max_steps=1000, params=None, chunk_vars=4_000_000, rows_per_instance=4096,
                  seed=7):
    params = params or solve_params()
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    stats = dict(sat=0, converged=0, instances=len(cnfs))
    chunk, nv = [], 0
    t0 = time.time()

    def flush():
        X, y, st = label_chunk(chunk, restarts, max_steps, params, seed, rows_per_instance, rng)
        xs.append(X)
        ys.append(y)
        stats["sat"] += st["sat"]
        stats["converged"] += st["converged"]
        log(f"labelled {stats['converged']} / {stats['instances']} instances "
            f"({stats['sat']} satisfied), {time.time() - t0:.0f} s")

    for c in cnfs:
        if chunk and nv + c.num_vars > chunk_vars:
            flush()
            chunk, nv = [], 0
        chunk.append(c)
        nv += c.num_vars
    if chunk:
        flush()
    return np.concatenate(xs), np.concatenate(ys), stats


# --------------------------------------------------------------------------
# training on the GPU
# --------------------------------------------------------------------------

def train(X: np.ndarray, y: np.ndarray, epochs: int = 3, batch: int = 16384, lr: float = 2e-3,
          seed: int = 11, device: int = 0, params: np.ndarray | None = None):
    """Adam on minibatches of (X, y) with the library's training kernels;
    torch holds the device buffers.  Returns (params, loss history)."""
    import torch

    dev = torch.device("cuda", device)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(X.shape[0])
    Xd = torch.from_numpy(np.ascontiguousarray(X[perm])).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(y[perm])).to(dev)
    net = tsat.Mlp(init_params(seed) if params is None else params, device=device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    n = X.shape[0]
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    hist = []
    step = 0
    for ep in range(epochs):
        off = int(rng.integers(0, batch)) if n > 2 * batch else 0
        for b in range(steps_per_epoch):
            i0 = (off + b * batch) % max(1, n - batch + 1)
            B = min(batch, n - i0)
            # cosine decay of the step size over the whole run
            cur = lr * 0.5 * (1 + np.cos(np.pi * step / total))
            net.train_step_dev(Xd[i0].data_ptr(), yd[i0:].data_ptr(), None, B, cur, stream)
            step += 1
            if step % 200 == 0 or step == total:
                _, loss = net.get_grad()
                hist.append((step, loss))
                log(f"epoch {ep} step {step}/{total} loss {loss:.4f}")
    out = net.get_params()
    net.close()
    return out, hist


def accuracy(params: np.ndarray, X: np.ndarray, y: np.ndarray, device: int = 0) -> float:
    """Fraction of rows where the proposal's more likely value is the label."""
    import torch

    dev = torch.device("cuda", device)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    pr = torch.empty(X.shape[0], device=dev)
    net = tsat.Mlp(params, device=device)
    net.forward_dev(Xd.data_ptr(), X.shape[0], None, pr.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize(dev)
    net.close()
    return float(((pr.cpu().numpy() > 0.5) == (y > 0.5)).mean())


# --------------------------------------------------------------------------
# learned versus random start
# --------------------------------------------------------------------------

def solve_params():
    """The search setting the proposal is trained and compared under."""
    return tsat.default_params(norm_mode=tsat.MODE_NONE, tau=2.0)


def majority_proposal(cnfs) -> np.ndarray:
    """Per variable (of the union of the instances, in load order), the
    Laplace-smoothed fraction of its occurrences that are positive: its most
    likely value is the majority polarity vote.  The baseline that shows
    what the network adds beyond the polarity counts among its features."""
    out = []
    for c in (cnfs if isinstance(cnfs, (list, tuple)) else [cnfs]):
        v = np.abs(c.lits) - 1
        pos = np.bincount(v[c.lits > 0], minlength=c.num_vars)
        neg = np.bincount(v[c.lits < 0], minlength=c.num_vars)
        out.append((pos + 1.0) / (pos + neg + 2.0))
    return np.concatenate(out).astype(np.float32)


ARMS = ("random", "majority", "learned")


def run_arm(cnf, arm: str, restarts: int, max_steps: int, seed: int, params, weights=None, device: int = 0):
    s = tsat.Solver(device=device, params=params)
    s.load(cnf)
    net = None
    if arm == "random":
        s.init_batch(restarts, seed=seed)
    elif arm == "majority":
        s.init_from_proposal(restarts, seed=seed, p_true=majority_proposal(cnf))
    elif arm == "learned":
        net = tsat.Mlp(weights, device=device)
        s.propose(net, want_host=False)
        s.init_from_proposal(restarts, seed=seed)
    else:
        raise ValueError(arm)
    sat0, _ = s.check()
    s.set_graph(True)
    t0 = time.perf_counter()
    r = s.step(max_steps, stop_on_sat=True)
    wall = time.perf_counter() - t0
    st = s.instance_status()[0]
    hz = s.device_clock_hz()
    out = dict(arm=arm, seed=seed, start_unsat=int(cnf.num_clauses - np.max(sat0)),
               steps_to_sat=r.first_sat_step, steps_to_99=r.first_converged_step,
               time_to_sat_s=((st["sat_ticks"] - st["start_ticks"]) / hz) if r.first_sat_step >= 0 else None,
               best_unsat=int(cnf.num_clauses - r.best_sat_count), steps_done=r.steps_done, wall_s=wall)
    if net is not None:
        net.close()
    s.close()
    return out


def compare(weights: np.ndarray, V: int = 100_000, ratio: float = 4.1, restarts: int = 128, max_steps: int = 3600,
            seeds=(1, 2, 3), instance_seed: int = 990_001, params=None, device: int = 0) -> dict:
    """Steps and time to all-SAT from the random, the majority-vote and the
    learned start on one held-out planted instance (same seeds for every
    arm)."""
    params = params or solve_params()
    cnf = gen.planted_ksat(V, int(round(ratio * V)), 3, seed=instance_seed)
    runs = []
    for sd in seeds:
        for arm in ARMS:
            runs.append(run_arm(cnf, arm, restarts, max_steps, sd, params, weights, device))
            log(json.dumps(runs[-1]))

    def summary(arm):
        rs = [r for r in runs if r["arm"] == arm]
        solved = [r for r in rs if r["steps_to_sat"] >= 0]
        med = lambda k, xs: float(np.median([x[k] for x in xs])) if xs else None  # noqa: E731
        return dict(solved=len(solved), runs=len(rs), median_steps_to_sat=med("steps_to_sat", solved),
                    median_time_to_sat_s=med("time_to_sat_s", solved),
                    median_steps_to_99=med("steps_to_99", [r for r in rs if r["steps_to_99"] >= 0]),
                    median_start_unsat=med("start_unsat", rs), median_best_unsat=med("best_unsat", rs))

    return dict(workload=f"held-out planted 3-SAT V={V}, C={int(round(ratio * V))}, {restarts} restarts, "
                         f"none-mode tau={params.tau}, cap {max_steps} steps",
                random=summary("random"), majority=summary("majority"), learned=summary("learned"), runs=runs)


def censored_percentile(values, n_total: int, q: float):
    """q-th percentile over n_total runs of which only len(values) have an
    observed value (the others ran past the cap: larger than every observed
    value); None when that order statistic is censored."""
    if n_total <= 0:
        return None
    k = max(1, int(np.ceil(q / 100.0 * n_total)))
    xs = np.sort(np.asarray(values, dtype=np.float64))
    return float(xs[k - 1]) if k <= xs.size else None


HELDOUT_CHECKPOINTS = (0, 25, 50, 100, 150, 200, 400, 800, 1600, 2400, 3600)


def evaluate_heldout(weights: np.ndarray, count: int = 20, V: int = 100_000, ratio: float = 4.1,
                     restarts: int = 128, max_steps: int = 3600, seed0: int = 20_000, init_seed: int = 1,
                     params=None, checkpoints=HELDOUT_CHECKPOINTS, device: int = 0) -> dict:
    """The random, majority-vote and learned starts on `count` held-out
    planted 3-SAT instances (V variables, ratio*V clauses, seeds seed0 + j),
    solved as one batch per arm: every instance freezes on its first
    satisfying candidate.  Per arm: steps and time to all-SAT (the learned
    arm's time includes its features and network, shared equally by the
    instances), censored at the step cap; steps to the 99% hand-off; and the
    lowest unsatisfied-clause count reached by each checkpoint (median over
    the instances)."""
    params = params or solve_params()
    C = int(round(ratio * V))
    cnfs = [gen.planted_ksat(V, C, 3, seed=seed0 + j) for j in range(count)]
    cps = sorted(set(int(c) for c in checkpoints if 0 <= c <= max_steps) | {max_steps})
    out = dict(workload=f"{count} held-out planted 3-SAT instances V={V}, C={C} (seeds {seed0}..{seed0 + count - 1}), "
                        f"{restarts} restarts, none-mode tau={params.tau}, cap {max_steps} steps, one batch per arm",
               checkpoints=cps)
    for arm in ARMS:
        s = tsat.Solver(device=device, params=params)
        s.load_batch(cnfs)
        net = None
        t0 = time.perf_counter()
        if arm == "random":
            s.init_batch(restarts, seed=init_seed)
        elif arm == "majority":
            s.init_from_proposal(restarts, seed=init_seed, p_true=majority_proposal(cnfs))
        else:
            net = tsat.Mlp(weights, device=device)
            s.propose(net, want_host=False)
            s.init_from_proposal(restarts, seed=init_seed)
        sat0, _ = s.check()  # synchronizes: the start is in place
        t_start = time.perf_counter() - t0
        unsat = C - sat0.reshape(count, restarts).max(axis=1)
        best = unsat.astype(np.int64).copy()
        curve = [float(np.median(best))]
        s.set_graph(True)
        done = 0
        for cp in cps[1:]:
            s.step(cp - done, stop_on_sat=True)
            done = cp
            st = s.instance_status()
            now = np.array([0 if x["first_sat_step"] >= 0 else x["num_clauses"] - x["best_sat_count"] for x in st])
            best = np.minimum(best, now)
            curve.append(float(np.median(best)))
            log(f"{arm}: step {cp}, solved {sum(x['first_sat_step'] >= 0 for x in st)}/{count}, "
                f"median best unsat {curve[-1]:.0f}")
        st = s.instance_status()
        hz = s.device_clock_hz()
        share = t_start / count if arm != "random" else 0.0
        sat_steps = [x["first_sat_step"] for x in st if x["first_sat_step"] >= 0]
        sat_times = [(x["sat_ticks"] - x["start_ticks"]) / hz + share for x in st if x["first_sat_step"] >= 0]
        s99 = [x["first_converged_step"] for x in st if x["first_converged_step"] >= 0]
        if net is not None:
            net.close()
        s.close()
        out[arm] = dict(
            solved=len(sat_steps), instances=count, censored=len(sat_steps) < count,
            p50_steps_to_sat=censored_percentile(sat_steps, count, 50),
            p90_steps_to_sat=censored_percentile(sat_steps, count, 90),
            p50_time_to_sat_s=censored_percentile(sat_times, count, 50),
            reached_99=len(s99), p50_steps_to_99=censored_percentile(s99, count, 50),
            median_start_unsat=float(np.median(unsat)), start_s=t_start,
            min_unsat_vs_step=curve)
    return out


def compare_batch(weights: np.ndarray, count: int = 400, vmin: int = 200, vmax: int = 1000, ratio: float = 4.0,
                  restarts: int = 32, max_steps: int = 3000, seed: int = 770_000, params=None,
                  device: int = 0) -> dict:
    """Steps to all-SAT per instance from the random, the majority-vote and
    the learned start, on a batch of small held-out planted instances solved
    together (each freezes on its first satisfying candidate).  Reports the
    solved counts and, over the instances the random and the learned start
    both solve, the median steps to SAT and how often each is faster."""
    params = params or solve_params()
    rng = np.random.default_rng(seed)
    Vs = np.exp(rng.uniform(np.log(vmin), np.log(vmax), size=count)).astype(int)
    cnfs = [gen.planted_ksat(int(v), int(round(ratio * v)), 3, seed=seed + j) for j, v in enumerate(Vs)]
    steps = {}
    for arm in ARMS:
        s = tsat.Solver(device=device, params=params)
        s.load_batch(cnfs)
        net = None
        if arm == "random":
            s.init_batch(restarts, seed=1)
        elif arm == "majority":
            s.init_from_proposal(restarts, seed=1, p_true=majority_proposal(cnfs))
        else:
            net = tsat.Mlp(weights, device=device)
            s.propose(net, want_host=False)
            s.init_from_proposal(restarts, seed=1)
        s.set_graph(True)
        s.step(max_steps, stop_on_sat=True)
        steps[arm] = np.array([x["first_sat_step"] for x in s.instance_status()])
        if net is not None:
            net.close()
        s.close()
    r, l = steps["random"], steps["learned"]
    both = (r >= 0) & (l >= 0)
    med = lambda x: float(np.median(x)) if x.size else None  # noqa: E731
    return dict(workload=f"{count} held-out planted 3-SAT instances, V log-uniform in [{vmin}, {vmax}], "
                         f"C = {ratio} V, {restarts} restarts, none-mode tau={params.tau}, cap {max_steps} steps",
                random=dict(solved=int((r >= 0).sum()), median_steps_to_sat=med(r[r >= 0])),
                majority=dict(solved=int((steps["majority"] >= 0).sum()),
                              median_steps_to_sat=med(steps["majority"][steps["majority"] >= 0])),
                learned=dict(solved=int((l >= 0).sum()), median_steps_to_sat=med(l[l >= 0])),
                both_solved=int(both.sum()), median_steps_both=dict(random=med(r[both]), learned=med(l[both])),
                learned_faster=int((l[both] < r[both]).sum()), random_faster=int((r[both] < l[both]).sum()))


def save_weights(path: str, params: np.ndarray, meta: dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), meta=np.array(json.dumps(meta)))


def load_weights(path: str = DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(str(z["meta"]))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--instances", type=int, default=5000)
    t.add_argument("--vmin", type=int, default=20_000)
    t.add_argument("--vmax", type=int, default=100_000)
    t.add_argument("--restarts", type=int, default=32)
    t.add_argument("--max-steps", type=int, default=1000)
    t.add_argument("--rows-per-instance", type=int, default=4096)
    t.add_argument("--epochs", type=int, default=3)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    c = sub.add_parser("compare")
    c.add_argument("--weights", default=DEFAULT_WEIGHTS)
    c.add_argument("--V", type=int, default=100_000)
    c.add_argument("--restarts", type=int, default=128)
    c.add_argument("--max-steps", type=int, default=3600)
    c.add_argument("--seeds", type=int, nargs="+", default=[1, 2, 3])
    args = ap.parse_args(argv)
    if args.cmd == "train":
        t0 = time.time()
        log(f"generating {args.instances} instances")
        cnfs = corpus(args.instances, vmin=args.vmin, vmax=args.vmax, workers=args.workers)
        t_gen = time.time() - t0
        X, y, stats = build_dataset(cnfs, args.restarts, args.max_steps, rows_per_instance=args.rows_per_instance)
        del cnfs
        t_lab = time.time() - t0 - t_gen
        n_val = max(1, X.shape[0] // 20)
        params, hist = train(X[n_val:], y[n_val:], epochs=args.epochs, lr=args.lr)
        acc = accuracy(params, X[:n_val], y[:n_val])
        meta = dict(instances=args.instances, vmin=args.vmin, vmax=args.vmax, restarts=args.restarts,
                    max_steps=args.max_steps, rows=int(X.shape[0]), label_stats=stats, epochs=args.epochs,
                    lr=args.lr, final_loss=hist[-1][1] if hist else None, val_accuracy=acc,
                    label_mean=float(y.mean()), gen_s=t_gen, label_s=t_lab, train_s=time.time() - t0 - t_gen - t_lab)
        save_weights(args.out, params, meta)
        print(json.dumps(meta))
    else:
        params, meta = load_weights(args.weights)
        out = compare(params, V=args.V, restarts=args.restarts, max_steps=args.max_steps, seeds=args.seeds)
        out["training"] = meta
        print(json.dumps(out))


if __name__ == "__main__":
    main()
