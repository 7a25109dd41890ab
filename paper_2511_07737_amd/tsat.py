"""Python binding of the gfx950 gradient-guided SAT library (C-ABI of ``include/tsat.h``).

Argument marshalling only: every step of the method runs in the HIP
library ``libtsat.so`` built in-tree by ``paper_2511_07737_amd.build``.  If the
library is missing, importing its functions raises immediately; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtsat.so")
_lib = None

OK = 0
E_ARG, E_PARSE, E_OOM, E_HIP, E_STATE, E_NUMERIC = -1, -2, -3, -4, -5, -6
MODE_NONE, MODE_MEAN = 0, 1
MAX_WIDTH = 32
MAX_STEP_N = 1024

_P = ct.c_void_p
_i32, _i64, _u64, _f32, _f64 = ct.c_int32, ct.c_int64, ct.c_uint64, ct.c_float, ct.c_double


class TsatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tsat error {code}: {msg}")
        self.code = code


class LaunchConfig(ct.Structure):
    _fields_ = [("fwd_target_blocks", ct.c_int32), ("var_blocks_per_cu", ct.c_int32), ("pure_group", ct.c_int32),
                ("clause_planes", ct.c_int32), ("window_gather", ct.c_int32), ("fwd_ms", ct.c_double),
                ("var_ms", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Params(ct.Structure):
    _fields_ = [
        ("tau", _f64), ("lr0", _f64), ("lr_decay", _f64), ("lr_min", _f64),
        ("beta1", _f64), ("beta2", _f64), ("eps", _f64), ("weight_decay", _f64),
        ("converge_frac", _f64),
        ("decay_every", _i32), ("restart_every", _i32), ("norm_mode", _i32), ("k_partial", _i32),
        ("mix", _i32), ("reserved", _i32),
    ]


class Config(ct.Structure):
    _fields_ = [("device", _i32), ("reserved", _i32), ("stream", _P), ("params", Params)]


class _Report(ct.Structure):
    _fields_ = [
        ("steps_done", _i64), ("first_sat_step", _i64), ("first_converged_step", _i64),
        ("best_sat_count", _i64), ("next_step", _i64), ("loss", _f64),
        ("best_candidate", _i32), ("sat_candidate", _i32), ("nonfinite", _i32), ("reserved", _i32),
    ]


class _InstStatus(ct.Structure):
    _fields_ = [
        ("first_sat_step", _i64), ("first_converged_step", _i64), ("best_sat_count", _i64),
        ("num_clauses", _i64), ("loss", _f64), ("start_ticks", _u64), ("sat_ticks", _u64),
        ("conv_ticks", _u64),
        ("best_candidate", _i32), ("sat_candidate", _i32), ("frozen", _i32), ("num_vars", _i32),
    ]


class _CnfInfo(ct.Structure):
    _fields_ = [
        ("num_vars", _i32), ("max_width", _i32), ("num_clauses", _i64), ("num_lits", _i64),
        ("num_empty", _i64), ("num_dup_removed", _i64), ("num_tautologies", _i64),
        ("width_count", _i64 * (MAX_WIDTH + 1)),
    ]


@dataclass
class Report:
    steps_done: int
    first_sat_step: int
    first_converged_step: int
    best_sat_count: int
    next_step: int
    loss: float
    best_candidate: int
    sat_candidate: int
    nonfinite: int


# (name, restype, argtypes) for every exported entry point
_SIGS = [
    ("tsat_last_error", ct.c_char_p, []),
    ("tsat_version", _i32, []),
    ("tsat_default_params", _i32, [ct.POINTER(Params)]),
    ("tsat_cnf_info_of", _i32, [_i32, _i64, _P, ct.POINTER(_CnfInfo)]),
    ("tsat_dimacs_read", _i32, [ct.c_char_p, ct.POINTER(_i32), ct.POINTER(_i64), _P, _i64]),
    ("tsat_create", _i32, [ct.POINTER(Config), ct.POINTER(_P)]),
    ("tsat_destroy", None, [_P]),
    ("tsat_load_cnf", _i32, [_P, _i32, _i64, _P]),
    ("tsat_load_dimacs", _i32, [_P, ct.c_char_p]),
    ("tsat_load_cnf_batch", _i32, [_P, _i32, _P, _P, _P]),
    ("tsat_num_instances", _i32, [_P]),
    ("tsat_num_vars", _i32, [_P]),
    ("tsat_set_graph", _i32, [_P, _i32]),
    ("tsat_get_instance_status", _i32, [_P, _i32, _i32, ct.POINTER(_InstStatus)]),
    ("tsat_device_clock_hz", _i32, [_P, ct.POINTER(_f64)]),
    ("tsat_get_witness_instance", _i32, [_P, _i32, _P, ct.POINTER(_i32)]),
    ("tsat_init_batch", _i32, [_P, _i32, _u64, _P]),
    ("tsat_step", _i32, [_P, _i32, ct.POINTER(Params), _i32, ct.POINTER(_Report)]),
    ("tsat_check", _i32, [_P, _P, _P]),
    ("tsat_check_bits", _i32, [_P, _P, _i32, _P, _P]),
    ("tsat_get_assignment", _i32, [_P, _i32, _P]),
    ("tsat_get_witness", _i32, [_P, _P, ct.POINTER(_i32)]),
    ("tsat_extract_partial", _i32, [_P, _i32, _i32, _P, _P, _P]),
    ("tsat_num_candidates", _i32, [_P]),
    ("tsat_max_width", _i32, [_P]),
    ("tsat_set_logits", _i32, [_P, _P]),
    ("tsat_get_logits", _i32, [_P, _P]),
    ("tsat_set_state", _i32, [_P, _P, _P, _P, _i64]),
    ("tsat_get_state", _i32, [_P, _P, _P, _P, ct.POINTER(_i64)]),
    ("tsat_get_bits", _i32, [_P, _P]),
    ("tsat_eval", _i32, [_P, ct.POINTER(Params), _P, _P, ct.POINTER(_f64)]),
    ("tsat_get_grad", _i32, [_P, ct.POINTER(Params), _P, _P]),
    ("tsat_pack_dev", _i32, [_P, _P, _i32, _P, _P]),
    ("tsat_fwd_dev", _i32, [_P, _P, _i32, _f32, _P, _P, _P]),
    ("tsat_fwd_dev_noalloc", _i32, [_P, _P, _i32, _f32, _P, _P, _P]),
    ("tsat_bwd_dev", _i32, [_P, _P, _i32, _f32, _P, _P, _P]),
    ("tsat_bwd_scatter_dev", _i32, [_P, _P, _i32, _f32, _P, _P, _P]),
    ("tsat_binarize_dev", _i32, [_P, _P, _i32, _i32, _P, _P, _P, _P]),
    ("tsat_get_adam_origin", _i32, [_P, _P]),
    ("tsat_set_adam_origin", _i32, [_P, _i64]),
    ("tsat_norm_backward_dev", _i32, [_P, _P, _P, _i32, _i32, _P, _P]),
    ("tsat_loss_dev", _i32, [_P, _P, _i32, _f32, _i32, _P, _P, _P, _P]),
    ("tsat_loss_backward_dev", _i32, [_P, _P, _i32, _f32, _i32, _P, _P, _P, _P]),
    ("tsat_set_timing", _i32, [_P, _i32]),
    ("tsat_get_timing", _i32, [_P, ct.POINTER(_f64), ct.POINTER(_i32)]),
    ("tsat_copy_calibrate", _i32, [_P, _i64, ct.POINTER(_f64)]),
    ("tsat_stream_calibrate", _i32, [_P, _i64, _i32, _i32, ct.POINTER(_f64)]),
    ("tsat_set_literal_rows", _i32, [_P, _i32]),
    ("tsat_get_launch_config", _i32, [_P, ct.POINTER(LaunchConfig)]),
    ("tsat_set_launch_config", _i32, [_P, ct.POINTER(LaunchConfig)]),
    ("tsat_autotune", _i32, [_P, _i32, _P, ct.POINTER(LaunchConfig), ct.POINTER(_i32)]),
    ("tsat_get_features", _i32, [_P, _P]),
    ("tsat_features_dev", _i32, [_P, _P, _P]),
    ("tsat_mlp_create", _i32, [_i32, _P, ct.POINTER(_P)]),
    ("tsat_mlp_destroy", None, [_P]),
    ("tsat_mlp_set_params", _i32, [_P, _P]),
    ("tsat_mlp_get_params", _i32, [_P, _P]),
    ("tsat_mlp_get_grad", _i32, [_P, _P, _P]),
    ("tsat_mlp_step_count", _i64, [_P]),
    ("tsat_mlp_forward_dev", _i32, [_P, _P, _i64, _P, _P, _P]),
    ("tsat_mlp_train_step_dev", _i32, [_P, _P, _P, _P, _i64, _f32, _P]),
    ("tsat_propose", _i32, [_P, _P, _P]),
    ("tsat_init_from_proposal", _i32, [_P, _i32, ct.c_uint64, _P]),
]


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2511_07737_amd.build.build()")
        # torch ships its own HIP runtime under the same soname as the system
        # one: whichever is loaded first serves the whole process, and torch
        # does not see the GPU through the other.  Load torch's first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ct.CDLL(_LIB_PATH)
        for name, rt, args in _SIGS:
            f = getattr(L, name)
            f.restype = rt
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise TsatError(rc, lib().tsat_last_error().decode(errors="replace"))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def last_error() -> str:
    return lib().tsat_last_error().decode(errors="replace")


def version() -> int:
    return int(lib().tsat_version())


def default_params(**kw) -> Params:
    p = Params()
    _check(lib().tsat_default_params(ct.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def cnf_info_of(num_vars: int, stream) -> dict:
    s = np.ascontiguousarray(stream, dtype=np.int32)
    info = _CnfInfo()
    _check(lib().tsat_cnf_info_of(int(num_vars), int(s.size), _ptr(s), ct.byref(info)))
    d = {f: getattr(info, f) for f, _ in _CnfInfo._fields_ if f != "width_count"}
    d["width_count"] = list(info.width_count)
    return d


def dimacs_read(path: str):
    V, n = _i32(), _i64()
    _check(lib().tsat_dimacs_read(path.encode(), ct.byref(V), ct.byref(n), None, 0))
    buf = np.empty(max(n.value, 1), dtype=np.int32)
    _check(lib().tsat_dimacs_read(path.encode(), ct.byref(V), ct.byref(n), _ptr(buf), n.value))
    return int(V.value), buf[: n.value]


class Solver:
    """One solver on one device (see ``include/tsat.h``)."""

    def __init__(self, device: int = 0, stream: int | None = None, params: Params | None = None):
        cfg = Config()
        cfg.device = device
        cfg.stream = stream
        cfg.params = params if params is not None else default_params()
        h = _P()
        _check(lib().tsat_create(ct.byref(cfg), ct.byref(h)))
        self._h = h
        self.V = 0
        self.N = 0
        self._lit_rows = 0  # requested for the next batch
        self.rows = 0       # logit rows of the current batch (V, or 2V with literal rows)

    # lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().tsat_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # loading ------------------------------------------------------------
    def load_cnf(self, num_vars: int, stream) -> None:
        s = np.ascontiguousarray(stream, dtype=np.int32)
        _check(lib().tsat_load_cnf(self._h, int(num_vars), int(s.size), _ptr(s)))
        self.V = int(num_vars)
        self.N = 0
        self._lit_rows = 0

    def load(self, cnf) -> None:
        """Load a ``gen.CNF``."""
        self.load_cnf(cnf.num_vars, cnf.dimacs_stream())

    def load_dimacs(self, path: str) -> None:
        _check(lib().tsat_load_dimacs(self._h, path.encode()))
        V, _ = dimacs_read(path)
        self.V = V
        self.N = 0
        self._lit_rows = 0

    def load_batch(self, cnfs) -> None:
        """Load a list of ``gen.CNF`` instances as one batch."""
        streams = [c.dimacs_stream() for c in cnfs]
        nv = np.array([c.num_vars for c in cnfs], dtype=np.int32)
        off = np.zeros(len(cnfs) + 1, dtype=np.int64)
        off[1:] = np.cumsum([s.size for s in streams])
        lits = np.concatenate(streams).astype(np.int32) if streams else np.zeros(0, dtype=np.int32)
        _check(lib().tsat_load_cnf_batch(self._h, len(cnfs), _ptr(nv), _ptr(off), _ptr(lits)))
        self.V = int(lib().tsat_num_vars(self._h))
        self.N = 0
        self._lit_rows = 0

    @property
    def num_instances(self) -> int:
        return int(lib().tsat_num_instances(self._h))

    def set_graph(self, enable: bool) -> None:
        _check(lib().tsat_set_graph(self._h, 1 if enable else 0))

    def instance_status(self, first: int = 0, count: int | None = None) -> list[dict]:
        n = self.num_instances - first if count is None else count
        arr = (_InstStatus * max(n, 1))()
        _check(lib().tsat_get_instance_status(self._h, int(first), int(n), arr))
        return [{f: getattr(arr[i], f) for f, _ in _InstStatus._fields_} for i in range(n)]

    def device_clock_hz(self) -> float:
        hz = _f64()
        _check(lib().tsat_device_clock_hz(self._h, ct.byref(hz)))
        return float(hz.value)

    def get_witness_instance(self, inst: int, num_vars: int):
        out = np.empty(num_vars, dtype=np.uint8)
        c = _i32()
        _check(lib().tsat_get_witness_instance(self._h, int(inst), _ptr(out), ct.byref(c)))
        return out, int(c.value)

    @property
    def max_width(self) -> int:
        return int(lib().tsat_max_width(self._h))

    def set_literal_rows(self, enable: bool) -> None:
        """Independent literal rows (2V logit rows) from the next init_batch on."""
        _check(lib().tsat_set_literal_rows(self._h, int(bool(enable))))
        self._lit_rows = int(bool(enable))
        self.N = 0

    def init_batch(self, n: int, seed: int = 0, init_logits: np.ndarray | None = None) -> None:
        rows = (2 if self._lit_rows else 1) * self.V
        lg = None
        if init_logits is not None:
            lg = np.ascontiguousarray(init_logits, dtype=np.float32)
            if lg.shape != (rows, n):
                raise ValueError(f"init_logits must have shape {(rows, n)}")
        _check(lib().tsat_init_batch(self._h, int(n), int(seed) & ((1 << 64) - 1), _ptr(lg)))
        self.N = int(n)
        self.rows = rows

    # launch shapes -------------------------------------------------------
    def launch_config(self) -> LaunchConfig:
        c = LaunchConfig()
        _check(lib().tsat_get_launch_config(self._h, ct.byref(c)))
        return c

    def set_launch_config(self, fwd_target_blocks=None, var_blocks_per_cu=None, pure_group=None,
                          clause_planes=None, window_gather=None) -> None:
        c = self.launch_config()
        if clause_planes is not None:
            c.clause_planes = int(clause_planes)
        if window_gather is not None:
            c.window_gather = int(window_gather)
        if fwd_target_blocks is not None:
            c.fwd_target_blocks = int(fwd_target_blocks)
        if var_blocks_per_cu is not None:
            c.var_blocks_per_cu = int(var_blocks_per_cu)
        if pure_group is not None:
            c.pure_group = int(pure_group)
        _check(lib().tsat_set_launch_config(self._h, ct.byref(c)))

    def autotune(self, iters: int = 3, params: Params | None = None):
        """Pick the fastest launch shapes on real iterations; returns (config, iterations used)."""
        c = LaunchConfig()
        used = _i32()
        _check(lib().tsat_autotune(self._h, int(iters), ct.byref(params) if params is not None else None,
                                   ct.byref(c), ct.byref(used)))
        return c, int(used.value)

    # learned proposal ---------------------------------------------------
    def get_features(self) -> np.ndarray:
        X = np.empty((self.V, MLP_FEATURES), dtype=np.float32)
        _check(lib().tsat_get_features(self._h, _ptr(X)))
        return X

    def features_dev(self, X_ptr: int, stream: int | None = None) -> None:
        _check(lib().tsat_features_dev(self._h, X_ptr, stream))

    def propose(self, mlp: "Mlp", want_host: bool = True) -> np.ndarray | None:
        p = np.empty(self.V, dtype=np.float32) if want_host else None
        _check(lib().tsat_propose(self._h, mlp.handle, _ptr(p)))
        return p

    def init_from_proposal(self, n: int, seed: int = 0, p_true: np.ndarray | None = None) -> None:
        pp = None
        if p_true is not None:
            pp = np.ascontiguousarray(p_true, dtype=np.float32)
            if pp.shape != (self.V,):
                raise ValueError(f"p_true must have shape {(self.V,)}")
        _check(lib().tsat_init_from_proposal(self._h, int(n), int(seed) & ((1 << 64) - 1), _ptr(pp)))
        self.N = int(n)
        self.rows = self.V

    # solving ------------------------------------------------------------
    def step(self, max_steps: int = 1, params: Params | None = None, stop_on_sat: bool | int = False,
             raise_numeric: bool = True) -> Report:
        """stop_on_sat: False/0 run all steps; True/1 freeze instances on a
        satisfying candidate; 2 also freeze them at convergence (hand-off)."""
        r = _Report()
        mode = 2 if stop_on_sat == 2 else (1 if stop_on_sat else 0)
        rc = lib().tsat_step(self._h, int(max_steps), ct.byref(params) if params is not None else None,
                             mode, ct.byref(r))
        if rc != OK and not (rc == E_NUMERIC and not raise_numeric):
            _check(rc)
        return Report(*[getattr(r, f) for f, _ in _Report._fields_ if f != "reserved"])

    def check(self):
        ni = self.num_instances
        sat = np.empty((ni, self.N), dtype=np.int64)
        ok = np.empty((ni, self.N), dtype=np.uint8)
        _check(lib().tsat_check(self._h, _ptr(sat), _ptr(ok)))
        return (sat[0], ok[0]) if ni == 1 else (sat, ok)

    def check_bits(self, packed: np.ndarray, n: int):
        p = np.ascontiguousarray(packed, dtype=np.uint64)
        W = (n + 63) // 64
        if p.shape != (self.V, W):
            raise ValueError(f"packed must have shape {(self.V, W)}")
        ni = self.num_instances
        sat = np.empty((ni, n), dtype=np.int64)
        ok = np.empty((ni, n), dtype=np.uint8)
        _check(lib().tsat_check_bits(self._h, _ptr(p), int(n), _ptr(sat), _ptr(ok)))
        return (sat[0], ok[0]) if ni == 1 else (sat, ok)

    def get_assignment(self, cand: int) -> np.ndarray:
        out = np.empty(self.V, dtype=np.uint8)
        _check(lib().tsat_get_assignment(self._h, int(cand), _ptr(out)))
        return out

    def get_witness(self):
        out = np.empty(self.V, dtype=np.uint8)
        c = _i32()
        _check(lib().tsat_get_witness(self._h, _ptr(out), ct.byref(c)))
        return out, int(c.value)

    def extract_partial(self, max_cands: int, k: int = 0):
        if k <= 0:
            k = max(20, -(-self.V // 10000))
        ids = np.empty(max_cands, dtype=np.int32)
        lits = np.empty((max_cands, k), dtype=np.int32)
        sat = np.empty(max_cands, dtype=np.int64)
        _check(lib().tsat_extract_partial(self._h, int(max_cands), int(k), _ptr(ids), _ptr(lits), _ptr(sat)))
        return ids, lits, sat

    # state --------------------------------------------------------------
    def set_logits(self, theta: np.ndarray) -> None:
        t = np.ascontiguousarray(theta, dtype=np.float32)
        _check(lib().tsat_set_logits(self._h, _ptr(t)))

    def get_logits(self) -> np.ndarray:
        out = np.empty((self.rows, self.N), dtype=np.float32)
        _check(lib().tsat_get_logits(self._h, _ptr(out)))
        return out

    def set_state(self, theta, m=None, v=None, t: int = 0) -> None:
        th = np.ascontiguousarray(theta, dtype=np.float32)
        mm = None if m is None else np.ascontiguousarray(m, dtype=np.float32)
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float32)
        _check(lib().tsat_set_state(self._h, _ptr(th), _ptr(mm), _ptr(vv), int(t)))

    def get_state(self):
        th = np.empty((self.rows, self.N), dtype=np.float32)
        m = np.empty_like(th)
        v = np.empty_like(th)
        t = _i64()
        _check(lib().tsat_get_state(self._h, _ptr(th), _ptr(m), _ptr(v), ct.byref(t)))
        return th, m, v, int(t.value)

    def get_adam_origin(self) -> int:
        t0 = _i64()
        _check(lib().tsat_get_adam_origin(self._h, ct.byref(t0)))
        return int(t0.value)

    def set_adam_origin(self, origin: int) -> None:
        _check(lib().tsat_set_adam_origin(self._h, int(origin)))

    def get_bits(self) -> np.ndarray:
        """Value rows [V][W], or every literal row [2V][W] with literal rows on."""
        out = np.empty((self.rows, (self.N + 63) // 64), dtype=np.uint64)
        _check(lib().tsat_get_bits(self._h, _ptr(out)))
        return out

    def eval(self, params: Params | None = None):
        K1 = self.max_width + 1
        ni = self.num_instances
        hist = np.empty((ni, self.N, K1), dtype=np.uint32)
        S = np.empty((ni, self.N), dtype=np.float64)
        loss = _f64()
        _check(lib().tsat_eval(self._h, ct.byref(params) if params is not None else None, _ptr(hist), _ptr(S),
                               ct.byref(loss)))
        if ni == 1:
            return hist[0], S[0], float(loss.value)
        return hist, S, float(loss.value)

    def get_grad(self, params: Params | None = None):
        U = np.empty((self.rows, self.N), dtype=np.float32)
        g = np.empty_like(U)
        _check(lib().tsat_get_grad(self._h, ct.byref(params) if params is not None else None, _ptr(U), _ptr(g)))
        return U, g

    # device-pointer API (integer addresses) --------------------------------
    def pack_dev(self, assign_ptr: int, n: int, bits_ptr: int, stream: int | None = None) -> None:
        _check(lib().tsat_pack_dev(self._h, assign_ptr, int(n), bits_ptr, stream))

    def fwd_dev(self, bits_ptr: int, n: int, tau: float, S_ptr: int | None, hist_ptr: int | None,
                stream: int | None = None) -> None:
        _check(lib().tsat_fwd_dev(self._h, bits_ptr, int(n), float(tau), S_ptr, hist_ptr, stream))

    def fwd_dev_noalloc(self, bits_ptr: int, n: int, tau: float, S_ptr: int | None, hist_ptr: int | None,
                        stream: int | None = None) -> None:
        _check(lib().tsat_fwd_dev_noalloc(self._h, bits_ptr, int(n), float(tau), S_ptr, hist_ptr, stream))

    def bwd_dev(self, bits_ptr: int, n: int, tau: float, dS_ptr: int, U_ptr: int, stream: int | None = None) -> None:
        _check(lib().tsat_bwd_dev(self._h, bits_ptr, int(n), float(tau), dS_ptr, U_ptr, stream))

    def bwd_scatter_dev(self, bits_ptr: int, n: int, tau: float, dS_ptr: int, U_ptr: int,
                        stream: int | None = None) -> None:
        _check(lib().tsat_bwd_scatter_dev(self._h, bits_ptr, int(n), float(tau), dS_ptr, U_ptr, stream))

    def binarize_dev(self, theta_ptr: int, n: int, mode: int, bits_ptr: int | None, assign_ptr: int | None,
                     mu_ptr: int | None, stream: int | None = None) -> None:
        _check(lib().tsat_binarize_dev(self._h, theta_ptr, int(n), int(mode), bits_ptr, assign_ptr, mu_ptr, stream))

    def norm_backward_dev(self, theta_ptr: int, dA_ptr: int, n: int, mode: int, g_ptr: int,
                          stream: int | None = None) -> None:
        _check(lib().tsat_norm_backward_dev(self._h, theta_ptr, dA_ptr, int(n), int(mode), g_ptr, stream))

    def loss_dev(self, theta_ptr: int, n: int, tau: float, mode: int, loss_ptr: int, S_ptr: int | None,
                 bits_ptr: int | None, stream: int | None = None) -> None:
        _check(lib().tsat_loss_dev(self._h, theta_ptr, int(n), float(tau), int(mode), loss_ptr, S_ptr, bits_ptr,
                                   stream))

    def loss_backward_dev(self, theta_ptr: int, n: int, tau: float, mode: int, dloss_ptr: int | None, g_ptr: int,
                          U_ptr: int | None, stream: int | None = None) -> None:
        _check(lib().tsat_loss_backward_dev(self._h, theta_ptr, int(n), float(tau), int(mode), dloss_ptr, g_ptr,
                                            U_ptr, stream))

    # timing ---------------------------------------------------------------
    def set_timing(self, enable: bool) -> None:
        _check(lib().tsat_set_timing(self._h, 1 if enable else 0))

    def get_timing(self):
        ms = (_f64 * 3)()
        it = _i32()
        _check(lib().tsat_get_timing(self._h, ms, ct.byref(it)))
        return list(ms), int(it.value)

    def stream_calibrate(self, nbytes: int, kind: int, reps: int = 10) -> float:
        """Average ms of a bandwidth reference kernel over arrays of nbytes
        (kind 0: copy; 1: three arrays in place, 16-byte accesses; 2: the same
        with the update kernels' 4-byte row pattern)."""
        ms = _f64()
        _check(lib().tsat_stream_calibrate(self._h, int(nbytes), int(kind), int(reps), ct.byref(ms)))
        return float(ms.value)

    def copy_calibrate(self, nbytes: int) -> float:
        """Run one plain device copy of nbytes (read + write); returns its ms."""
        ms = _f64()
        _check(lib().tsat_copy_calibrate(self._h, int(nbytes), ct.byref(ms)))
        return float(ms.value)


MLP_FEATURES = 16
MLP_HIDDEN = 128
MLP_NUM_PARAMS = 18817


class Mlp:
    """The learned-proposal network on one device (see ``include/tsat.h``).
    Device-pointer calls take raw addresses (e.g. ``tensor.data_ptr()``) and a
    HIP stream handle (None: the null stream)."""

    def __init__(self, params: np.ndarray, device: int = 0):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NUM_PARAMS,):
            raise ValueError(f"params must have shape ({MLP_NUM_PARAMS},)")
        h = _P()
        _check(lib().tsat_mlp_create(int(device), _ptr(p), ct.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().tsat_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: np.ndarray) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NUM_PARAMS,):
            raise ValueError(f"params must have shape ({MLP_NUM_PARAMS},)")
        _check(lib().tsat_mlp_set_params(self._h, _ptr(p)))

    def get_params(self) -> np.ndarray:
        p = np.empty(MLP_NUM_PARAMS, dtype=np.float32)
        _check(lib().tsat_mlp_get_params(self._h, _ptr(p)))
        return p

    def get_grad(self):
        g = np.empty(MLP_NUM_PARAMS, dtype=np.float32)
        loss = np.empty(1, dtype=np.float32)
        _check(lib().tsat_mlp_get_grad(self._h, _ptr(g), _ptr(loss)))
        return g, float(loss[0])

    def step_count(self) -> int:
        return int(lib().tsat_mlp_step_count(self._h))

    def forward_dev(self, X_ptr: int, B: int, logits_ptr: int | None, probs_ptr: int | None,
                    stream: int | None = None) -> None:
        _check(lib().tsat_mlp_forward_dev(self._h, X_ptr, int(B), logits_ptr, probs_ptr, stream))

    def train_step_dev(self, X_ptr: int, y_ptr: int, w_ptr: int | None, B: int, lr: float,
                       stream: int | None = None) -> None:
        _check(lib().tsat_mlp_train_step_dev(self._h, X_ptr, y_ptr, w_ptr, int(B), float(lr), stream))


def pack_bits(values: np.ndarray) -> np.ndarray:
    """Host helper: uint8/bool [V][N] -> uint64 [V][ceil(N/64)] (candidate c = bit c%64 of word c/64)."""
    v = np.asarray(values).astype(np.uint64)
    V, N = v.shape
    W = (N + 63) // 64
    pad = np.zeros((V, W * 64), dtype=np.uint64)
    pad[:, :N] = v
    return (pad.reshape(V, W, 64) << np.arange(64, dtype=np.uint64)).sum(axis=2, dtype=np.uint64)


def unpack_bits(packed: np.ndarray, n: int) -> np.ndarray:
    """Host helper: uint64 [V][W] -> uint8 [V][n]."""
    p = np.asarray(packed, dtype=np.uint64)
    V, W = p.shape
    bits = (p[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(V, W * 64)[:, :n].astype(np.uint8)
