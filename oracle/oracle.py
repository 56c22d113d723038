"""ctypes wrapper of the plain CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product path (the HIP library and its binding)
never touches it.  See ``oracle.c`` for what each routine follows in the
paper and which readings it takes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

SIGMA_AUTO, SIGMA_FP = 0, 1
STOP_COND, STOP_OMEGA, STOP_PAUSED = 1, 2, 3
STREAM_ADS, STREAM_CALIB = 0, 1
MLP_PARAMS = 4481


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (FP contraction off)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-pthread",
            "-shared", "-fPIC", "-o", tmp, os.path.join(HERE, "oracle.c"), "-lm",
        ])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int32), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p)]


class SampleInfo(C.Structure):
    _fields_ = [("s", C.c_int32), ("t", C.c_int32), ("d", C.c_int32), ("w", C.c_int32),
                ("side", C.c_int32), ("steps", C.c_int32), ("meet_size", C.c_int32),
                ("fp_mode", C.c_int32), ("edges", C.c_int64), ("draws", C.c_uint64),
                ("sigma_st_int", C.c_uint64), ("sigma_st", C.c_double), ("sigma_exp", C.c_int32),
                ("visited", C.c_int32)]


class RunOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("stream", C.c_uint64), ("eps", C.c_double),
                ("omega", C.c_double), ("epoch", C.c_uint64), ("sigma_mode", C.c_int),
                ("start_epoch", C.c_int32), ("stop_after_epochs", C.c_int32)]


class RunResult(C.Structure):
    _fields_ = [("tau", C.c_uint64), ("epochs", C.c_int32), ("reason", C.c_int32),
                ("edges", C.c_int64)]


class CheckInfo(C.Structure):
    _fields_ = [("max_f", C.c_double), ("max_g", C.c_double), ("min_abs_margin", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.orc_draw.restype = u64
        L.orc_draw.argtypes = [u64, u64, u64, u64]
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_pair.argtypes = [u64, u64, u64, i32, vp, vp]
        L.orc_ws_create.restype = vp
        L.orc_ws_create.argtypes = [i32]
        L.orc_ws_free.argtypes = [vp]
        L.orc_sample_path.restype = C.c_int
        L.orc_sample_path.argtypes = [vp, vp, u64, u64, u64, C.c_int, vp, vp]
        L.orc_sample_fixed.restype = C.c_int
        L.orc_sample_fixed.argtypes = [vp, vp, u64, u64, u64, C.c_int, i32, i32, vp, vp]
        for fn in (L.orc_f, L.orc_g):
            fn.restype = dbl
            fn.argtypes = [dbl, dbl, dbl, dbl]
        L.orc_omega.restype = dbl
        L.orc_omega.argtypes = [i64, dbl, dbl]
        L.orc_omega_bracket.restype = dbl
        L.orc_omega_bracket.argtypes = [i64, i64, dbl, dbl]
        L.orc_vd_bracket.argtypes = [vp, vp, vp]
        L.orc_exact_vd.restype = i64
        L.orc_exact_vd.argtypes = [vp]
        L.orc_eccentricity.restype = i32
        L.orc_eccentricity.argtypes = [vp, i32]
        L.orc_check.restype = C.c_int
        L.orc_check.argtypes = [i32, vp, u64, dbl, dbl, vp, vp, vp]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32]
        L.orc_count.restype = C.c_int
        L.orc_count.argtypes = [vp, u64, u64, u64, u64, C.c_int, vp, vp]
        L.orc_run_mt.restype = C.c_int
        L.orc_run_mt.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, C.c_int]
        L.orc_count_mt.restype = C.c_int
        L.orc_count_mt.argtypes = [vp, u64, u64, u64, u64, C.c_int, vp, vp, C.c_int]
        L.orc_calibrate_mt.restype = C.c_int
        L.orc_calibrate_mt.argtypes = [vp, u64, dbl, dbl, C.c_int, vp, vp, vp, vp, C.c_int]
        L.orc_neglog.argtypes = [i32, vp, vp]
        L.orc_alloc_constant.restype = dbl
        L.orc_alloc_constant.argtypes = [i32, vp, dbl]
        L.orc_alloc_delta.argtypes = [i32, vp, dbl, dbl, dbl, vp, vp]
        L.orc_calibrate.restype = C.c_int
        L.orc_calibrate.argtypes = [vp, u64, dbl, dbl, C.c_int, vp, vp, vp, vp]
        L.orc_brandes.argtypes = [vp, vp]
        L.orc_features.argtypes = [vp, vp]
        L.orc_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.orc_prior_from_output.argtypes = [i64, vp, dbl, vp]
        L.orc_mlp_loss_grad.restype = dbl
        L.orc_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp]
        L.orc_adam_step.argtypes = [vp, vp, vp, vp, i64, i64, dbl, dbl, dbl, dbl]
        L.orc_mlp_init.argtypes = [u64, vp]
        L.orc_batch_rows.argtypes = [u64, u64, i32, i64, vp]
        L.orc_mlp_train.argtypes = [vp, vp, i64, i32, i32, dbl, i32, u64, vp, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Graph:
    """Holds the CSR arrays alive for the C side."""

    def __init__(self, g):
        self.n = int(g.n)
        self.row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(g.col_idx, dtype=np.int32)
        self._s = _Graph(self.n, self.row_ptr.ctypes.data, self.col_idx.ctypes.data)

    @property
    def ref(self):
        return C.byref(self._s)


def as_graph(g) -> Graph:
    return g if isinstance(g, Graph) else Graph(g)


# ------------------------------------------------------------------ RNG


def philox_block(key0: int, key1: int, ctr) -> np.ndarray:
    key = np.array([key0, key1], dtype=np.uint64)
    c = np.array(ctr, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(key), _p(c), _p(out))
    return out


def draw(seed: int, stream: int, sample: int, j: int) -> int:
    return int(lib().orc_draw(seed, stream, sample, j))


def pair(seed: int, stream: int, sample: int, n: int):
    s, t = C.c_int32(), C.c_int32()
    lib().orc_pair(seed, stream, sample, n, C.byref(s), C.byref(t))
    return s.value, t.value


# -------------------------------------------------------------- samples


class Sampler:
    """One workspace, many samples (avoids re-allocating per sample)."""

    def __init__(self, g, seed: int = 1, stream: int = STREAM_ADS, sigma_mode: int = SIGMA_AUTO):
        self.g = as_graph(g)
        self.seed, self.stream, self.sigma_mode = seed, stream, sigma_mode
        self.ws = lib().orc_ws_create(self.g.n)
        self.buf = np.zeros(self.g.n + 1, dtype=np.int32)

    def __del__(self):
        if getattr(self, "ws", None):
            lib().orc_ws_free(self.ws)
            self.ws = None

    def sample(self, i: int):
        """Returns (path s..t as an int32 array, SampleInfo)."""
        info = SampleInfo()
        rc = lib().orc_sample_path(self.g.ref, self.ws, self.seed, self.stream, i,
                                   self.sigma_mode, _p(self.buf), C.byref(info))
        if rc != 0:
            raise RuntimeError(f"oracle sample {i} failed: {rc}")
        return self.buf[: info.d + 1].copy(), info

    def sample_fixed(self, i: int, s: int, t: int):
        """Sample i, but for the given pair (s, t) instead of a drawn one."""
        info = SampleInfo()
        rc = lib().orc_sample_fixed(self.g.ref, self.ws, self.seed, self.stream, i,
                                    self.sigma_mode, s, t, _p(self.buf), C.byref(info))
        if rc != 0:
            raise RuntimeError(f"oracle sample {i} failed: {rc}")
        return self.buf[: info.d + 1].copy(), info


def host_threads() -> int:
    """Threads the host lets this process run at once: its CPU affinity,
    capped by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def count(g, seed: int, stream: int, first: int, cnt: int, sigma_mode: int = SIGMA_AUTO,
          threads: int = 1):
    g = as_graph(g)
    c = np.zeros(g.n, dtype=np.uint32)
    edges = C.c_int64()
    if threads > 1:
        rc = lib().orc_count_mt(g.ref, seed, stream, first, cnt, sigma_mode, _p(c), C.byref(edges), threads)
    else:
        rc = lib().orc_count(g.ref, seed, stream, first, cnt, sigma_mode, _p(c), C.byref(edges))
    if rc != 0:
        raise RuntimeError(f"oracle count failed: {rc}")
    return c, edges.value


# ------------------------------------------------------------ stop rule


def f(bt, L, omega, tau) -> float:
    return lib().orc_f(bt, L, omega, tau)


def g(bt, L, omega, tau) -> float:
    return lib().orc_g(bt, L, omega, tau)


def fg_arrays(c: np.ndarray, tau: int, omega: float, LL: np.ndarray, LU: np.ndarray):
    fo = np.array([lib().orc_f(float(ci) / tau, float(l), omega, float(tau)) for ci, l in zip(c, LL)])
    go = np.array([lib().orc_g(float(ci) / tau, float(l), omega, float(tau)) for ci, l in zip(c, LU)])
    return fo, go


def omega(vd: int, eps: float, delta: float) -> float:
    return lib().orc_omega(vd, eps, delta)


def omega_bracket(vd_lo: int, vd_hi: int, eps: float, delta: float) -> float:
    return lib().orc_omega_bracket(vd_lo, vd_hi, eps, delta)


def vd_bracket(g):
    g = as_graph(g)
    lo, hi = C.c_int64(), C.c_int64()
    lib().orc_vd_bracket(g.ref, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def exact_vd(g) -> int:
    return int(lib().orc_exact_vd(as_graph(g).ref))


def eccentricity(g, v: int) -> int:
    return int(lib().orc_eccentricity(as_graph(g).ref, v))


def check(c: np.ndarray, tau: int, omega_: float, eps: float, LL, LU):
    ci = CheckInfo()
    c = np.ascontiguousarray(c, dtype=np.uint32)
    LL = np.ascontiguousarray(LL, dtype=np.float64)
    LU = np.ascontiguousarray(LU, dtype=np.float64)
    ok = lib().orc_check(len(c), _p(c), tau, omega_, eps, _p(LL), _p(LU), C.byref(ci))
    return bool(ok), ci


def run(g, *, seed=1, eps=0.01, omega_: float, epoch=1024, LL, LU, sigma_mode=SIGMA_AUTO,
        stream=STREAM_ADS, start_epoch=0, stop_after_epochs=0, c_init=None, max_epochs=4096,
        threads=1):
    """Epoch loop to the stop rule.  Returns dict with counters and per-epoch
    info.  threads > 1: every epoch's samples split over that many threads
    (same result)."""
    g = as_graph(g)
    LL = np.ascontiguousarray(LL, dtype=np.float64)
    LU = np.ascontiguousarray(LU, dtype=np.float64)
    c = np.zeros(g.n, dtype=np.uint32) if c_init is None else np.array(c_init, dtype=np.uint32)
    opts = RunOpts(seed, stream, eps, omega_, epoch, sigma_mode, start_epoch, stop_after_epochs)
    res = RunResult()
    per = (CheckInfo * max_epochs)()
    if threads > 1:
        rc = lib().orc_run_mt(g.ref, C.byref(opts), _p(LL), _p(LU), _p(c), C.byref(res), per, max_epochs,
                              threads)
    else:
        rc = lib().orc_run(g.ref, C.byref(opts), _p(LL), _p(LU), _p(c), C.byref(res), per, max_epochs)
    if rc != 0:
        raise RuntimeError(f"oracle run failed: {rc}")
    k = min(res.epochs, max_epochs)
    return dict(c=c, tau=res.tau, epochs=res.epochs, reason=res.reason, edges=res.edges,
                max_f=np.array([per[i].max_f for i in range(start_epoch, k)]),
                max_g=np.array([per[i].max_g for i in range(start_epoch, k)]),
                min_margin=np.array([per[i].min_abs_margin for i in range(start_epoch, k)]))


# ---------------------------------------------------------- calibration


def alloc_constant(prior: np.ndarray, delta: float) -> float:
    prior = np.ascontiguousarray(prior, dtype=np.float64)
    return lib().orc_alloc_constant(len(prior), _p(prior), delta)


def alloc_delta(prior: np.ndarray, Cc: float, delta: float, beta: float = 1e-3):
    prior = np.ascontiguousarray(prior, dtype=np.float64)
    LL = np.zeros(len(prior))
    LU = np.zeros(len(prior))
    lib().orc_alloc_delta(len(prior), _p(prior), Cc, delta, beta, _p(LL), _p(LU))
    return LL, LU


def calibrate(g, *, seed=1, omega_: float, delta=0.1, sigma_mode=SIGMA_AUTO, threads=1):
    g = as_graph(g)
    cp = np.zeros(g.n, dtype=np.uint32)
    LL = np.zeros(g.n)
    LU = np.zeros(g.n)
    Cc = C.c_double()
    rc = lib().orc_calibrate_mt(g.ref, seed, omega_, delta, sigma_mode, _p(cp), C.byref(Cc), _p(LL), _p(LU),
                                threads)
    if rc != 0:
        raise RuntimeError(f"oracle calibration failed: {rc}")
    return dict(cprime=cp, C=Cc.value, LL=LL, LU=LU, tau0=int(np.ceil(omega_ / 100.0)))


def neglog(delta: np.ndarray) -> np.ndarray:
    """L = -ln(delta) per vertex, computed by the oracle (libm log in FP64)."""
    d = np.ascontiguousarray(delta, dtype=np.float64)
    L = np.zeros(len(d))
    lib().orc_neglog(len(d), _p(d), _p(L))
    return L


def uniform_delta(n: int, delta: float):
    """delta_L = delta_U = 0.999 delta / (4n): a valid allocation (sum below delta / 2)."""
    L = np.full(n, -np.log(0.999 * delta / (4.0 * n)))
    return L, L.copy()


# ---------------------------------------------------------------- exact


def brandes(g) -> np.ndarray:
    g = as_graph(g)
    bc = np.zeros(g.n)
    lib().orc_brandes(g.ref, _p(bc))
    return bc


# --------------------------------------------------------------- learned


def features(g) -> np.ndarray:
    g = as_graph(g)
    x = np.zeros((g.n, 3))
    lib().orc_features(g.ref, _p(x))
    return x


def mlp_forward(params: np.ndarray, x: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(len(x))
    lib().orc_mlp_forward(_p(p), _p(x), len(x), _p(y))
    return y


def prior_from_output(y: np.ndarray, omega_: float) -> np.ndarray:
    """Learned prior b = e^y - 1/omega clamped to [0, 1]."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    pr = np.zeros(len(y))
    lib().orc_prior_from_output(len(y), _p(y), omega_, _p(pr))
    return pr


def mlp_loss_grad(params: np.ndarray, x: np.ndarray, target: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(target, dtype=np.float64)
    gr = np.zeros(MLP_PARAMS)
    loss = lib().orc_mlp_loss_grad(_p(p), _p(x), _p(t), len(x), _p(gr))
    return loss, gr


def adam_step(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays."""
    lib().orc_adam_step(_p(params), _p(grad), _p(m), _p(v), len(params), step, lr, b1, b2, eps)


def mlp_init(seed: int) -> np.ndarray:
    p = np.zeros(MLP_PARAMS)
    lib().orc_mlp_init(seed, _p(p))
    return p


def batch_rows(seed: int, step: int, batch: int, rows: int) -> np.ndarray:
    out = np.zeros(batch, dtype=np.int64)
    lib().orc_batch_rows(seed, step, batch, rows, _p(out))
    return out


def mlp_train(x: np.ndarray, y: np.ndarray, *, epochs: int, batch: int, lr: float, halve_every: int, seed: int):
    """FP64 training loop (initialisation, batches, Adam); returns (params, per-epoch losses)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    p = np.zeros(MLP_PARAMS)
    losses = np.zeros(epochs)
    lib().orc_mlp_train(_p(x), _p(y), len(y), epochs, batch, lr, halve_every, seed, _p(p), _p(losses))
    return p, losses
