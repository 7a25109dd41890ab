"""Seeded synthetic CNF instances and initial logits.

This module produces inputs only: instances (planted random k-SAT, a
community-structured power-law family, ragged multi-instance sets), the
N(0,1) initial logits, and enumerated candidate assignments for brute-force
checks.  It contains none of the solver's arithmetic (no binarization, no
clause counting, no loss, no gradient, no optimizer), so the GPU path and the
CPU oracle can both consume what it makes without sharing method code.

Every generator takes an integer seed and uses numpy's counter-based Philox
bit generator, so the same seed gives the same instance on any machine.

CNF convention: variables are numbered 1..V; a literal is +v or -v
(DIMACS).  ``CNF.offsets`` (int64, length C+1) delimits clauses inside
``CNF.lits`` (int32, length L).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CNF",
    "rng",
    "planted_ksat",
    "random_ksat",
    "structured",
    "ragged_set",
    "normal_logits",
    "enumerate_assignments",
    "width_pmf",
]


def rng(seed: int) -> np.random.Generator:
    """Philox4x32-10 stream keyed by ``seed``."""
    return np.random.Generator(np.random.Philox(key=int(seed) & ((1 << 64) - 1)))


@dataclass
class CNF:
    num_vars: int
    offsets: np.ndarray  # int64 [C+1]
    lits: np.ndarray  # int32 [L], signed 1-based
    planted: np.ndarray | None = None  # uint8 [V] hidden satisfying assignment
    meta: dict = field(default_factory=dict)

    @property
    def num_clauses(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def num_lits(self) -> int:
        return int(self.lits.shape[0])

    def clause(self, c: int) -> np.ndarray:
        return self.lits[self.offsets[c] : self.offsets[c + 1]]

    def widths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def dimacs_stream(self) -> np.ndarray:
        """Clauses as one int32 stream, each clause followed by a 0."""
        C = self.num_clauses
        out = np.zeros(self.num_lits + C, dtype=np.int32)
        w = self.widths()
        # position of each literal in the output = its index + clause index
        cid = np.repeat(np.arange(C, dtype=np.int64), w)
        out[np.arange(self.num_lits, dtype=np.int64) + cid] = self.lits
        return out

    @staticmethod
    def from_clauses(num_vars: int, clauses, planted=None) -> "CNF":
        offs = [0]
        flat = []
        for cl in clauses:
            flat.extend(int(x) for x in cl)
            offs.append(len(flat))
        return CNF(
            num_vars=int(num_vars),
            offsets=np.asarray(offs, dtype=np.int64),
            lits=np.asarray(flat, dtype=np.int32),
            planted=None if planted is None else np.asarray(planted, dtype=np.uint8),
        )

    def to_dimacs(self) -> str:
        lines = [f"p cnf {self.num_vars} {self.num_clauses}"]
        for c in range(self.num_clauses):
            lines.append(" ".join(str(int(x)) for x in self.clause(c)) + " 0")
        return "\n".join(lines) + "\n"


def _distinct_rows(g: np.random.Generator, n: int, k: int, hi: int) -> np.ndarray:
    """(n, k) int64 in [0, hi) with distinct entries in every row."""
    if k > hi:
        raise ValueError(f"cannot draw {k} distinct variables out of {hi}")
    out = g.integers(0, hi, size=(n, k), dtype=np.int64)
    if k == 1:
        return out
    while True:
        s = np.sort(out, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            return out
        out[bad] = g.integers(0, hi, size=(bad.size, k), dtype=np.int64)


def _literals_true(vars_: np.ndarray, pos: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Whether each literal (variable index, polarity) is true under z."""
    zv = z[vars_]
    return np.where(pos, zv == 1, zv == 0)


def planted_ksat(num_vars: int, num_clauses: int, k: int = 3, seed: int = 0, p_pos: float = 0.5) -> CNF:
    """Uniform random k-SAT with a planted solution.

    A hidden assignment z ~ Bern(0.5)^V is drawn first.  Each clause takes k
    distinct variables uniformly and positive polarity with probability
    ``p_pos``; the whole clause is redrawn until z satisfies it.
    """
    g = rng(seed)
    z = g.integers(0, 2, size=num_vars, dtype=np.uint8)
    out = np.empty((num_clauses, k), dtype=np.int32)
    todo = np.arange(num_clauses, dtype=np.int64)
    while todo.size:
        n = todo.size
        vs = _distinct_rows(g, n, k, num_vars)
        pos = g.random((n, k)) < p_pos
        ok = _literals_true(vs, pos, z).any(axis=1)
        lit = np.where(pos, vs + 1, -(vs + 1)).astype(np.int32)
        out[todo[ok]] = lit[ok]
        todo = todo[~ok]
    offs = np.arange(num_clauses + 1, dtype=np.int64) * k
    return CNF(num_vars, offs, out.reshape(-1), z, {"kind": "planted", "k": k, "seed": seed})


def random_ksat(num_vars: int, num_clauses: int, k: int = 3, seed: int = 0, p_pos: float = 0.5) -> CNF:
    """Uniform random k-SAT without a planted solution (distinct variables per clause)."""
    g = rng(seed)
    vs = _distinct_rows(g, num_clauses, k, num_vars)
    pos = g.random((num_clauses, k)) < p_pos
    lit = np.where(pos, vs + 1, -(vs + 1)).astype(np.int32)
    offs = np.arange(num_clauses + 1, dtype=np.int64) * k
    return CNF(num_vars, offs, lit.reshape(-1), None, {"kind": "random", "k": k, "seed": seed})


def width_pmf(kmin: int = 2, kmax: int = 12, exponent: float = 2.5) -> tuple[np.ndarray, np.ndarray]:
    ks = np.arange(kmin, kmax + 1)
    w = ks.astype(np.float64) ** (-exponent)
    return ks, w / w.sum()


def structured(
    num_vars: int,
    num_clauses: int,
    seed: int = 0,
    kmin: int = 2,
    kmax: int = 12,
    width_exp: float = 2.5,
    occ_exp: float = 2.2,
    communities: int = 64,
    p_intra: float = 0.9,
    p_pos: float = 0.5,
) -> CNF:
    """Community-structured planted CNF with power-law widths and occurrences.

    Clause width k on [kmin, kmax] with P(k) proportional to k^-width_exp.
    Variables are split into ``communities`` contiguous blocks; within a
    block a seeded permutation ranks the variables and rank r (1-based) is
    drawn with probability proportional to r^(-1/(occ_exp-1)) (the
    scale-free model of Ansotegui, Bonet and Levy).  Each literal slot takes
    its variable from the clause's home community with probability
    ``p_intra``, otherwise from a uniformly chosen other community.  The
    variables of one clause are distinct; polarity is positive with
    probability ``p_pos``; the clause is redrawn (slots and polarities) until
    the hidden assignment satisfies it.
    """
    g = rng(seed)
    z = g.integers(0, 2, size=num_vars, dtype=np.uint8)
    ks, pk = width_pmf(kmin, kmax, width_exp)
    if kmax > num_vars:
        raise ValueError("kmax exceeds the number of variables")
    widths = g.choice(ks, size=num_clauses, p=pk)
    bounds = (np.arange(communities + 1, dtype=np.int64) * num_vars) // communities
    sizes = np.diff(bounds)
    # rank -> variable, per community (a seeded permutation of its block)
    rank_to_var = np.empty(num_vars, dtype=np.int64)
    for c in range(communities):
        rank_to_var[bounds[c] : bounds[c + 1]] = bounds[c] + g.permutation(int(sizes[c]))
    alpha = 1.0 / (occ_exp - 1.0)
    cdfs = {}
    for s in np.unique(sizes):
        w = np.arange(1, int(s) + 1, dtype=np.float64) ** (-alpha)
        cdf = np.cumsum(w)
        cdfs[int(s)] = cdf / cdf[-1]
    home = g.integers(0, communities, size=num_clauses, dtype=np.int64)

    def draw_slots(h: np.ndarray, k: int) -> np.ndarray:
        n = h.shape[0]
        intra = g.random((n, k)) < p_intra
        other = (h[:, None] + g.integers(1, communities, size=(n, k), dtype=np.int64)) % communities
        comm = np.where(intra, h[:, None], other)
        u = g.random((n, k))
        rank = np.empty((n, k), dtype=np.int64)
        csz = sizes[comm]
        for s, cdf in cdfs.items():
            sel = csz == s
            if sel.any():
                rank[sel] = np.minimum(np.searchsorted(cdf, u[sel], side="right"), s - 1)
        return rank_to_var[bounds[comm] + rank]

    offs = np.zeros(num_clauses + 1, dtype=np.int64)
    offs[1:] = np.cumsum(widths)
    lits = np.empty(int(offs[-1]), dtype=np.int32)
    for k in ks:
        idx = np.nonzero(widths == k)[0]
        if idx.size == 0:
            continue
        k = int(k)
        todo = np.arange(idx.size, dtype=np.int64)
        res = np.empty((idx.size, k), dtype=np.int32)
        while todo.size:
            h = home[idx[todo]]
            vs = draw_slots(h, k)
            # redraw rows with repeated variables until every row is distinct
            while True:
                s = np.sort(vs, axis=1)
                bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
                if bad.size == 0:
                    break
                vs[bad] = draw_slots(h[bad], k)
            pos = g.random((todo.size, k)) < p_pos
            ok = _literals_true(vs, pos, z).any(axis=1)
            lit = np.where(pos, vs + 1, -(vs + 1)).astype(np.int32)
            res[todo[ok]] = lit[ok]
            todo = todo[~ok]
        starts = offs[idx]
        lits[(starts[:, None] + np.arange(k)[None, :]).reshape(-1)] = res.reshape(-1)
    return CNF(num_vars, offs, lits, z, {"kind": "structured", "seed": seed})


def ragged_set(
    count: int = 1000,
    seed: int = 3000,
    vmin: int = 1000,
    vmax: int = 200000,
    ratio_lo: float = 3.8,
    ratio_hi: float = 4.2,
    k: int = 3,
) -> list[CNF]:
    """Planted k-SAT instances with V log-uniform in [vmin, vmax] and ratio uniform
    in [ratio_lo, ratio_hi]; instance j uses seed ``seed + j``."""
    return [ragged_instance(j, seed, vmin, vmax, ratio_lo, ratio_hi, k) for j in range(count)]


def ragged_instance(j: int, seed: int = 3000, vmin: int = 1000, vmax: int = 200000, ratio_lo: float = 3.8,
                    ratio_hi: float = 4.2, k: int = 3) -> CNF:
    """Instance j of ``ragged_set`` (drawn on its own, so sets can be built in parallel)."""
    g = rng(seed + j)
    V = int(round(math.exp(g.uniform(math.log(vmin), math.log(vmax)))))
    C = int(round(g.uniform(ratio_lo, ratio_hi) * V))
    return planted_ksat(V, C, k=k, seed=(seed + j) * 7919 + 1)


def normal_logits(num_vars: int, n: int, seed: int) -> np.ndarray:
    """float32 [V][N] logits drawn from N(0, 1)."""
    return rng(seed).standard_normal(size=(num_vars, n), dtype=np.float32)


def enumerate_assignments(n: int) -> np.ndarray:
    """All 2^n assignments of n variables, bit-packed as uint64 [n][ceil(2^n/64)].

    Candidate i assigns variable v the value of bit v of i.
    """
    total = 1 << n
    words = (total + 63) // 64
    cand = np.arange(total, dtype=np.uint64)
    out = np.zeros((n, words), dtype=np.uint64)
    for v in range(n):
        bits = ((cand >> np.uint64(v)) & np.uint64(1)).astype(np.uint8)
        padded = np.zeros(words * 64, dtype=np.uint64)
        padded[:total] = bits
        out[v] = (padded.reshape(words, 64) << np.arange(64, dtype=np.uint64)).sum(axis=1, dtype=np.uint64)
    return out
