"""FP64 CPU oracle of the gradient-guided SAT step (TurboSAT, arXiv 2511.07737).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark are the only callers.  The product path
(the HIP library and its Python binding) never imports this package.

Thin ctypes wrapper over ``liboracle.so`` (built from ``tsat_oracle.c`` by
``build()``).  Arrays are numpy; floating point is float64 throughout.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsat_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ct.CDLL(_LIB)
        P = ct.c_void_p
        i32, i64, dbl = ct.c_int32, ct.c_int64, ct.c_double
        L.orc_cnf_new.argtypes = [i32, i64, P, ct.POINTER(P)]
        L.orc_cnf_free.argtypes = [P]
        L.orc_cnf_free.restype = None
        for name, rt in (("orc_cnf_num_clauses", i64), ("orc_cnf_num_lits", i64),
                         ("orc_cnf_max_width", i32), ("orc_cnf_num_vars", i32)):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = rt
        L.orc_cnf_get.argtypes = [P, P, P]
        L.orc_binarize.argtypes = [i32, i32, P, i32, P, P]
        L.orc_result_matrix.argtypes = [P, i32, P, P]
        L.orc_histogram.argtypes = [P, i32, P, P]
        L.orc_check.argtypes = [P, i32, P, P, P]
        L.orc_smoothmin.argtypes = [i32, i32, P, dbl, P, P, P, P]
        L.orc_adjoint.argtypes = [P, i32, P, i32, P, P]
        L.orc_norm_backward.argtypes = [i32, i32, P, i32, P, P]
        L.orc_lr.argtypes = [i64, dbl, dbl, i32, i32, dbl]
        L.orc_lr.restype = dbl
        L.orc_adamw.argtypes = [i64, P, P, P, P, dbl, dbl, dbl, dbl, dbl, i64]
        L.orc_adamw.restype = None
        L.orc_step.argtypes = [P, i32, P, i64, P, P, P, P, P, P, P, P, P]
        L.orc_step_ex.argtypes = [P, i32, P, i32, i64, i64, P, P, P, P, P, P, P, P, P, P]
        L.orc_best_candidate.argtypes = [i32, i32, P]
        L.orc_best_candidate.restype = i32
        L.orc_mix.argtypes = [i32, i32, P, i32]
        L.orc_lit_histogram.argtypes = [P, i32, P, P]
        L.orc_lit_adjoint.argtypes = [P, i32, P, i32, P, P]
        L.orc_relaxed_S.argtypes = [P, i32, P, i32, dbl]
        L.orc_relaxed_S.restype = dbl
        L.orc_relaxed_fd.argtypes = [P, i32, P, i32, i32, dbl, dbl]
        L.orc_relaxed_fd.restype = dbl
        L.orc_relaxed_loss.argtypes = [P, i32, P, dbl]
        L.orc_relaxed_loss.restype = dbl
        L.orc_extract_partial.argtypes = [P, i32, P, P, P, i32, i32, P, P, P]
        L.orc_features.argtypes = [P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox4x32_10.restype = None
        L.orc_init_normal.argtypes = [i32, i32, ct.c_uint64, P]
        L.orc_init_proposal.argtypes = [i32, i32, ct.c_uint64, P, i32, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


class Params(ct.Structure):
    _fields_ = [
        ("tau", ct.c_double), ("lr0", ct.c_double), ("decay", ct.c_double), ("lr_min", ct.c_double),
        ("beta1", ct.c_double), ("beta2", ct.c_double), ("eps", ct.c_double), ("weight_decay", ct.c_double),
        ("every", ct.c_int32), ("restart", ct.c_int32), ("mode", ct.c_int32), ("mix", ct.c_int32),
    ]


MODE_NONE = 0
MODE_MEAN = 1


def default_params(**kw) -> Params:
    d = dict(tau=1.0, lr0=0.1, decay=0.1, lr_min=1e-15, beta1=0.9, beta2=0.999, eps=1e-8,
             weight_decay=1e-2, every=30, restart=360, mode=MODE_MEAN, mix=0)
    d.update(kw)
    return Params(**d)


class Cnf:
    """Oracle-side CNF (clauses de-duplicated by the oracle's own parser)."""

    def __init__(self, num_vars: int, stream: np.ndarray):
        stream = np.ascontiguousarray(stream, dtype=np.int32)
        h = ct.c_void_p()
        _check(lib().orc_cnf_new(int(num_vars), int(stream.size), _p(stream), ct.byref(h)), "cnf_new")
        self._h = h
        L = lib()
        self.V = int(L.orc_cnf_num_vars(h))
        self.C = int(L.orc_cnf_num_clauses(h))
        self.L = int(L.orc_cnf_num_lits(h))
        self.K = int(L.orc_cnf_max_width(h))

    @classmethod
    def from_gen(cls, cnf) -> "Cnf":
        return cls(cnf.num_vars, cnf.dimacs_stream())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_cnf_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def clauses(self):
        off = np.empty(self.C + 1, dtype=np.int64)
        lit = np.empty(max(self.L, 1), dtype=np.int32)
        _check(lib().orc_cnf_get(self._h, _p(off), _p(lit)), "cnf_get")
        return off, lit[: self.L]


def binarize(theta: np.ndarray, mode: int = MODE_MEAN):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    V, N = theta.shape
    b = np.empty((V, N), dtype=np.uint8)
    mu = np.empty(V, dtype=np.float64)
    _check(lib().orc_binarize(V, N, _p(theta), mode, _p(b), _p(mu)), "binarize")
    return b, mu


def result_matrix(cnf: Cnf, b: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint8)
    N = b.shape[1]
    R = np.empty((cnf.C, N), dtype=np.int32)
    _check(lib().orc_result_matrix(cnf.handle, N, _p(b), _p(R)), "result_matrix")
    return R


def histogram(cnf: Cnf, b: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint8)
    N = b.shape[1]
    H = np.empty((N, cnf.K + 1), dtype=np.int64)
    _check(lib().orc_histogram(cnf.handle, N, _p(b), _p(H)), "histogram")
    return H


def check(cnf: Cnf, b: np.ndarray):
    b = np.ascontiguousarray(b, dtype=np.uint8)
    N = b.shape[1]
    sat = np.empty(N, dtype=np.int64)
    ok = np.empty(N, dtype=np.uint8)
    _check(lib().orc_check(cnf.handle, N, _p(b), _p(sat), _p(ok)), "check")
    return sat, ok


def smoothmin(H: np.ndarray, tau: float = 1.0, dS: np.ndarray | None = None):
    H = np.ascontiguousarray(H, dtype=np.int64)
    N, K1 = H.shape
    S = np.empty(N, dtype=np.float64)
    table = np.empty((N, K1), dtype=np.float64)
    loss = ct.c_double()
    dS_arr = None if dS is None else np.ascontiguousarray(dS, dtype=np.float64)
    _check(lib().orc_smoothmin(N, K1 - 1, _p(H), float(tau), _p(dS_arr), _p(S), _p(table),
                               ct.cast(ct.byref(loss), ct.c_void_p)), "smoothmin")
    return S, table, float(loss.value)


def adjoint(cnf: Cnf, b: np.ndarray, table: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint8)
    table = np.ascontiguousarray(table, dtype=np.float64)
    N = b.shape[1]
    U = np.empty((cnf.V, N), dtype=np.float64)
    _check(lib().orc_adjoint(cnf.handle, N, _p(b), table.shape[1] - 1, _p(table), _p(U)), "adjoint")
    return U


def norm_backward(theta: np.ndarray, U: np.ndarray, mode: int = MODE_MEAN) -> np.ndarray:
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    V, N = theta.shape
    g = np.empty((V, N), dtype=np.float64)
    _check(lib().orc_norm_backward(V, N, _p(theta), mode, _p(U), _p(g)), "norm_backward")
    return g


def lr(t: int, p: Params | None = None) -> float:
    p = p or default_params()
    return float(lib().orc_lr(int(t), p.lr0, p.decay, p.every, p.restart, p.lr_min))


def adamw(theta, m, v, g, lr_, t, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-2):
    """In-place AdamW on float64 arrays; t is the 1-based step count."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_adamw(theta.size, _p(theta), _p(m), _p(v), _p(g), float(lr_), beta1, beta2, eps, wd, int(t))


def step(cnf: Cnf, theta, m, v, t: int, p: Params | None = None, t_reset: int = 0, literal_rows: bool = False):
    """One iteration from (theta, m, v) at 0-based index t (orc_step_ex).
    literal_rows: theta has 2V rows, one per literal (row 2v = x_v, 2v+1 =
    not x_v).  Returns a dict with the new state, the intermediate
    quantities and ``mixed`` (the best candidate of a mixing iteration, else -1)."""
    p = p or default_params()
    theta = np.array(theta, dtype=np.float64, order="C", copy=True)
    m = np.array(m, dtype=np.float64, order="C", copy=True)
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    rows, N = theta.shape
    b = np.empty((rows, N), dtype=np.uint8)
    H = np.empty((N, cnf.K + 1), dtype=np.int64)
    S = np.empty(N, dtype=np.float64)
    U = np.empty((rows, N), dtype=np.float64)
    g = np.empty((rows, N), dtype=np.float64)
    loss = ct.c_double()
    mixed = ct.c_int32(-1)
    _check(lib().orc_step_ex(cnf.handle, N, ct.byref(p), 2 if literal_rows else 1, int(t), int(t_reset), _p(theta),
                             _p(m), _p(v), _p(b), _p(H), _p(S), ct.cast(ct.byref(loss), ct.c_void_p), _p(U), _p(g),
                             ct.cast(ct.byref(mixed), ct.c_void_p)), "step")
    return dict(theta=theta, m=m, v=v, bits=b, H=H, S=S, loss=float(loss.value), U=U, g=g, mixed=int(mixed.value))


def best_candidate(H: np.ndarray) -> int:
    """Most satisfied clauses (fewest R = 0), the lower index on ties."""
    H = np.ascontiguousarray(H, dtype=np.int64)
    N, K1 = H.shape
    return int(lib().orc_best_candidate(N, K1 - 1, _p(H)))


def mix(theta: np.ndarray, istar: int) -> np.ndarray:
    """Assignment mixing into candidate istar (a new array)."""
    th = np.array(theta, dtype=np.float64, order="C", copy=True)
    rows, N = th.shape
    _check(lib().orc_mix(rows, N, _p(th), int(istar)), "mix")
    return th


def lit_histogram(cnf: Cnf, bl: np.ndarray) -> np.ndarray:
    """H[N][K+1] of independent literal rows bl [2V][N]."""
    bl = np.ascontiguousarray(bl, dtype=np.uint8)
    N = bl.shape[1]
    H = np.empty((N, cnf.K + 1), dtype=np.int64)
    _check(lib().orc_lit_histogram(cnf.handle, N, _p(bl), _p(H)), "lit_histogram")
    return H


def lit_adjoint(cnf: Cnf, bl: np.ndarray, table: np.ndarray) -> np.ndarray:
    """U2[2V][N]: dL/dA of every literal row (straight-through, +1)."""
    bl = np.ascontiguousarray(bl, dtype=np.uint8)
    table = np.ascontiguousarray(table, dtype=np.float64)
    N = bl.shape[1]
    U2 = np.empty((2 * cnf.V, N), dtype=np.float64)
    _check(lib().orc_lit_adjoint(cnf.handle, N, _p(bl), table.shape[1] - 1, _p(table), _p(U2)), "lit_adjoint")
    return U2


def relaxed_S(cnf: Cnf, x: np.ndarray, i: int, tau: float = 1.0) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_relaxed_S(cnf.handle, x.shape[1], _p(x), int(i), float(tau)))


def relaxed_fd(cnf: Cnf, x: np.ndarray, v: int, i: int, h: float = 1e-3, tau: float = 1.0) -> float:
    """(S~_i(x + h e_vi) - S~_i(x - h e_vi)) / (2h), free of cancellation in the column sums."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_relaxed_fd(cnf.handle, x.shape[1], _p(x), int(v), int(i), float(h), float(tau)))


def relaxed_loss(cnf: Cnf, x: np.ndarray, tau: float = 1.0) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_relaxed_loss(cnf.handle, x.shape[1], _p(x), float(tau)))


def extract_partial(cnf: Cnf, g, b, sat_count, max_cands: int, k: int):
    g = np.ascontiguousarray(g, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    sat_count = np.ascontiguousarray(sat_count, dtype=np.int64)
    N = g.shape[1]
    ids = np.empty(max_cands, dtype=np.int32)
    lits = np.empty((max_cands, k), dtype=np.int32)
    sat = np.empty(max_cands, dtype=np.int64)
    _check(lib().orc_extract_partial(cnf.handle, N, _p(g), _p(b), _p(sat_count), max_cands, k,
                                     _p(ids), _p(lits), _p(sat)), "extract_partial")
    return ids, lits, sat


def default_k(num_vars: int) -> int:
    """k = 0.01% of the variables, at least 20 (Sec. IV-B)."""
    return max(20, -(-num_vars // 10000))


NUM_FEATURES = 16


def features(cnf: Cnf) -> np.ndarray:
    """Per-variable features of the learned proposal, float64 [V][16] (reading R9)."""
    X = np.empty((cnf.V, NUM_FEATURES), dtype=np.float64)
    _check(lib().orc_features(cnf.handle, _p(X)), "features")
    return X


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def init_normal(V: int, N: int, seed: int) -> np.ndarray:
    th = np.empty((V, N), dtype=np.float32)
    _check(lib().orc_init_normal(int(V), int(N), int(seed), _p(th)), "init_normal")
    return th


def init_proposal(p_true: np.ndarray, N: int, seed: int, mode: int = MODE_MEAN) -> np.ndarray:
    p = np.ascontiguousarray(p_true, dtype=np.float32)
    th = np.empty((p.size, N), dtype=np.float32)
    _check(lib().orc_init_proposal(int(p.size), int(N), int(seed), _p(p), int(mode), _p(th)), "init_proposal")
    return th
