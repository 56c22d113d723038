"""Python binding of the gfx950 KADABRA library (``include/kadabra.h``).

Argument marshalling only: every step of the sampling path runs in the HIP
kernels of ``libkadabra_hip.so``.  Loading fails loudly when the library
has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkadabra_hip.so")

KAD_OK = 0
STATUS = {0: "KAD_OK", -1: "KAD_EINVAL", -2: "KAD_ENOMEM", -3: "KAD_EDEVICE",
          -4: "KAD_ENOTCONNECTED", -5: "KAD_ESTATE", -6: "KAD_EOVERFLOW"}
KAD_STREAM_ADS, KAD_STREAM_CALIB, KAD_STREAM_TUNE = 0, 1, 5
KAD_ALLOC_PLAIN, KAD_ALLOC_EXPLICIT, KAD_ALLOC_LEARNED = 0, 1, 2
KAD_SIGMA_AUTO, KAD_SIGMA_FP = 0, 1
KAD_STOP_NONE, KAD_STOP_COND, KAD_STOP_OMEGA = 0, 1, 2
KAD_VISITED_AUTO, KAD_VISITED_DENSE, KAD_VISITED_HASHED = 0, 1, 2
KAD_GRAPH_VALIDATE = 1
MLP_PARAMS = 4481
INFO_WIDTH = 14


class KadError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class kad_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("epsilon", C.c_double), ("delta", C.c_double),
                ("epoch_size", C.c_uint32), ("alloc_mode", C.c_int32),
                ("omega_override", C.c_double), ("sigma_mode", C.c_int32), ("slots", C.c_int32),
                ("visited_budget_bytes", C.c_uint64), ("epochs_in_flight", C.c_int32),
                ("use_graphs", C.c_int32), ("block_size", C.c_int32), ("timing", C.c_int32),
                ("pools", C.c_int32), ("exact_diameter", C.c_int32), ("visited_mode", C.c_int32),
                ("visited_log2", C.c_int32)]


class kad_result(C.Structure):
    _fields_ = [("tau", C.c_uint64), ("tau0", C.c_uint64), ("epochs", C.c_uint32),
                ("stop_reason", C.c_int32), ("omega", C.c_double), ("vd_lo", C.c_int64),
                ("vd_hi", C.c_int64), ("t_omega_ms", C.c_double), ("t_alloc_ms", C.c_double),
                ("t_ads_ms", C.c_double), ("t_total_ms", C.c_double),
                ("t_sample_kernel_ms", C.c_double), ("sample_launches", C.c_uint32),
                ("edges_scanned", C.c_int64), ("vertices_expanded", C.c_int64),
                ("vertices_visited", C.c_int64), ("pred_edges", C.c_int64),
                ("path_vertices", C.c_int64), ("fp_samples", C.c_int64), ("max_f", C.c_double),
                ("max_g", C.c_double), ("min_margin", C.c_double), ("epoch_size", C.c_uint32),
                ("slots", C.c_int32), ("samples_run", C.c_int64), ("block_size", C.c_int32),
                ("pools", C.c_int32), ("visited_mode", C.c_int32), ("visited_log2", C.c_int32),
                ("deferred", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class kad_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("lr_halve_every", C.c_int32), ("seed", C.c_uint64)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_vp, _i32, _i64, _u32, _u64, _dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
_P = C.POINTER
SIGNATURES = [
    ("kad_create", C.c_int, [C.c_int, _vp, _P(_vp)]),
    ("kad_destroy", None, [_vp]),
    ("kad_last_error", C.c_char_p, []),
    ("kad_graph_upload", C.c_int, [_vp, _i32, _i64, _vp, _vp, _u32, _P(_vp)]),
    ("kad_graph_free", None, [_vp]),
    ("kad_sampler_init", C.c_int, [_vp, _vp, _P(kad_opts), _P(_vp)]),
    ("kad_sampler_free", None, [_vp]),
    ("kad_sampler_reset", C.c_int, [_vp, _u64]),
    ("kad_set_delta", C.c_int, [_vp, _vp, _vp]),
    ("kad_set_mlp_weights", C.c_int, [_vp, _vp, _vp]),
    ("kad_step_epoch", C.c_int, [_vp, _P(C.c_int)]),
    ("kad_run_to_stop", C.c_int, [_vp, _P(kad_result)]),
    ("kad_fetch_counts", C.c_int, [_vp, _vp, _P(_u64)]),
    ("kad_fetch_btilde", C.c_int, [_vp, _vp]),
    ("kad_fetch_fg", C.c_int, [_vp, _vp, _vp]),
    ("kad_fetch_delta", C.c_int, [_vp, _vp, _vp]),
    ("kad_fetch_result", C.c_int, [_vp, _P(kad_result)]),
    ("kad_fetch_history", C.c_int, [_vp, _u32, _vp]),
    ("kad_fetch_calibration", C.c_int, [_vp, _vp, _P(_u64), _P(_dbl)]),
    ("kad_count_samples", C.c_int, [_vp, _u64, _u64, _u64, _vp]),
    ("kad_sample_paths", C.c_int, [_vp, _u64, _u64, _u32, _i32, _vp, _vp]),
    ("kad_count_samples_noalloc", C.c_int, [_vp, _vp, _u64, _u64, _u64, _u64, _i32, _vp]),
    ("kad_philox", C.c_int, [_vp, _u64, _u64, _u64, _u32, _u32, _vp]),
    ("kad_vd_bracket", C.c_int, [_vp, _vp, _P(_i64), _P(_i64)]),
    ("kad_omega", _dbl, [_i64, _i64, _dbl, _dbl]),
    ("kad_exact_vd", C.c_int, [_vp, _vp, _P(_i64), _P(_i32), _P(_i64)]),
    ("kad_features", C.c_int, [_vp, _vp, _vp, _vp]),
    ("kad_device_alloc", C.c_int, [_vp, C.c_size_t, _P(_vp)]),
    ("kad_device_free", C.c_int, [_vp, _vp]),
    ("kad_memcpy_h2d", C.c_int, [_vp, _vp, _vp, C.c_size_t]),
    ("kad_memcpy_d2h", C.c_int, [_vp, _vp, _vp, C.c_size_t]),
    ("kad_mlp_create", C.c_int, [_vp, _vp, _P(_vp)]),
    ("kad_mlp_free", None, [_vp]),
    ("kad_mlp_get_params", C.c_int, [_vp, _vp]),
    ("kad_mlp_loss_grad", C.c_int, [_vp, _vp, _vp, _i64, _P(C.c_float), _vp]),
    ("kad_mlp_train_step", C.c_int, [_vp, _vp, _vp, _i64, C.c_float, _P(C.c_float)]),
    ("kad_mlp_forward", C.c_int, [_vp, _vp, _i64, _vp, _vp]),
    ("kad_mlp_train", C.c_int, [_vp, _P(_vp), _P(_vp), _vp, _i32, _P(kad_train_opts), _vp, _vp, _vp]),
]


def lib():
    """Loads libkadabra_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != KAD_OK:
        raise KadError(st, lib().kad_last_error().decode())


def _p(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


# ------------------------------------------------------------ thin wrappers
# Each mirrors the C entry point of the same name.


def kad_create(device: int = 0, hip_stream: int | None = None):
    out = _vp()
    _check(lib().kad_create(device, hip_stream, C.byref(out)))
    return out


def kad_destroy(ctx):
    lib().kad_destroy(ctx)


def kad_graph_upload(ctx, row_ptr: np.ndarray, col_idx: np.ndarray, validate: bool = False):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    out = _vp()
    _check(lib().kad_graph_upload(ctx, len(rp) - 1, int(rp[-1]), _p(rp), _p(ci),
                                  KAD_GRAPH_VALIDATE if validate else 0, C.byref(out)))
    return out


def kad_graph_free(g):
    lib().kad_graph_free(g)


def make_opts(seed=1, epsilon=0.01, delta=0.1, epoch_size=0, alloc_mode=KAD_ALLOC_PLAIN,
              omega_override=0.0, sigma_mode=KAD_SIGMA_AUTO, slots=0, visited_budget_bytes=0,
              epochs_in_flight=0, use_graphs=0, block_size=0, timing=0, pools=0, exact_diameter=0,
              visited_mode=0, visited_log2=0) -> kad_opts:
    return kad_opts(seed, epsilon, delta, epoch_size, alloc_mode, omega_override, sigma_mode, slots,
                    visited_budget_bytes, epochs_in_flight, use_graphs, block_size, timing, pools, exact_diameter,
                    visited_mode, visited_log2)


def kad_sampler_init(ctx, g, opts: kad_opts):
    out = _vp()
    _check(lib().kad_sampler_init(ctx, g, C.byref(opts), C.byref(out)))
    return out


def kad_sampler_free(s):
    lib().kad_sampler_free(s)


def kad_sampler_reset(s, seed: int):
    _check(lib().kad_sampler_reset(s, seed))


def kad_set_delta(s, delta_L: np.ndarray, delta_U: np.ndarray):
    dl = np.ascontiguousarray(delta_L, dtype=np.float64)
    du = np.ascontiguousarray(delta_U, dtype=np.float64)
    _check(lib().kad_set_delta(s, _p(dl), _p(du)))


def kad_set_mlp_weights(s, params: np.ndarray, norm: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    nm = np.ascontiguousarray(norm, dtype=np.float32)
    _check(lib().kad_set_mlp_weights(s, _p(p), _p(nm)))


def kad_step_epoch(s) -> bool:
    stopped = C.c_int()
    _check(lib().kad_step_epoch(s, C.byref(stopped)))
    return bool(stopped.value)


def kad_run_to_stop(s) -> kad_result:
    r = kad_result()
    _check(lib().kad_run_to_stop(s, C.byref(r)))
    return r


def kad_fetch_counts(s, n: int):
    c = np.zeros(n, dtype=np.uint32)
    tau = _u64()
    _check(lib().kad_fetch_counts(s, _p(c), C.byref(tau)))
    return c, tau.value


def kad_fetch_btilde(s, n: int) -> np.ndarray:
    b = np.zeros(n)
    _check(lib().kad_fetch_btilde(s, _p(b)))
    return b


def kad_fetch_fg(s, n: int):
    f = np.zeros(n)
    g = np.zeros(n)
    _check(lib().kad_fetch_fg(s, _p(f), _p(g)))
    return f, g


def kad_fetch_delta(s, n: int):
    a = np.zeros(n)
    b = np.zeros(n)
    _check(lib().kad_fetch_delta(s, _p(a), _p(b)))
    return a, b


def kad_fetch_result(s) -> kad_result:
    r = kad_result()
    _check(lib().kad_fetch_result(s, C.byref(r)))
    return r


def kad_fetch_history(s, epochs: int) -> np.ndarray:
    h = np.zeros((max(epochs, 1), 4))
    _check(lib().kad_fetch_history(s, epochs, _p(h)))
    return h[:epochs]


def kad_fetch_calibration(s, n: int):
    c = np.zeros(n, dtype=np.uint32)
    tau0 = _u64()
    Cc = _dbl()
    _check(lib().kad_fetch_calibration(s, _p(c), C.byref(tau0), C.byref(Cc)))
    return c, tau0.value, Cc.value


def kad_count_samples(s, stream: int, first: int, count: int, n: int) -> np.ndarray:
    c = np.zeros(n, dtype=np.uint32)
    _check(lib().kad_count_samples(s, stream, first, count, _p(c)))
    return c


def kad_count_samples_noalloc(ctx, g, seed: int, stream: int, first: int, count: int, sigma_mode: int,
                              d_c: int):
    _check(lib().kad_count_samples_noalloc(ctx, g, seed, stream, first, count, sigma_mode, C.c_void_p(d_c)))


def kad_sample_paths(s, stream: int, first: int, count: int, max_len: int):
    paths = np.full((count, max_len), -1, dtype=np.int32)
    info = np.zeros((count, INFO_WIDTH), dtype=np.int64)
    _check(lib().kad_sample_paths(s, stream, first, count, max_len, _p(paths), _p(info)))
    return paths, info


def kad_philox(ctx, seed: int, stream: int, first: int, count: int, nwords: int) -> np.ndarray:
    out = np.zeros((count, nwords), dtype=np.uint64)
    _check(lib().kad_philox(ctx, seed, stream, first, count, nwords, _p(out)))
    return out


def kad_vd_bracket(ctx, g):
    lo, hi = _i64(), _i64()
    _check(lib().kad_vd_bracket(ctx, g, C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def kad_exact_vd(ctx, g):
    """Returns (VD, witness caller id, BFS runs)."""
    vd, w, nb = _i64(), _i32(), _i64()
    _check(lib().kad_exact_vd(ctx, g, C.byref(vd), C.byref(w), C.byref(nb)))
    return vd.value, w.value, nb.value


def kad_omega(vd_lo: int, vd_hi: int, eps: float, delta: float) -> float:
    return lib().kad_omega(vd_lo, vd_hi, eps, delta)


def kad_features(ctx, g, n: int) -> np.ndarray:
    out = np.zeros((n, 3), dtype=np.float32)
    _check(lib().kad_features(ctx, g, None, _p(out)))
    return out


def kad_features_device(ctx, g, d_out_ptr: int):
    _check(lib().kad_features(ctx, g, C.c_void_p(d_out_ptr), None))


def kad_device_alloc(ctx, nbytes: int) -> int:
    out = _vp()
    _check(lib().kad_device_alloc(ctx, nbytes, C.byref(out)))
    return out.value


def kad_device_free(ctx, d_ptr: int):
    _check(lib().kad_device_free(ctx, C.c_void_p(d_ptr)))


def kad_memcpy_h2d(ctx, d_dst: int, h_src: np.ndarray):
    a = np.ascontiguousarray(h_src)
    _check(lib().kad_memcpy_h2d(ctx, C.c_void_p(d_dst), _p(a), a.nbytes))


def kad_memcpy_d2h(ctx, h_dst: np.ndarray, d_src: int):
    assert h_dst.flags["C_CONTIGUOUS"]
    _check(lib().kad_memcpy_d2h(ctx, _p(h_dst), C.c_void_p(d_src), h_dst.nbytes))


class DeviceArray:
    """A host array copied into device memory owned by the library (no
    other HIP runtime involved).  .ptr is the device address."""

    def __init__(self, ctx: "Context", a: np.ndarray):
        self.ctx = ctx
        a = np.ascontiguousarray(a)
        self.shape, self.dtype, self.nbytes = a.shape, a.dtype, a.nbytes
        self.ptr = kad_device_alloc(ctx.h, a.nbytes)
        kad_memcpy_h2d(ctx.h, self.ptr, a)

    def numpy(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=self.dtype)
        kad_memcpy_d2h(self.ctx.h, out, self.ptr)
        return out

    def close(self):
        if self.ptr and self.ctx.h:
            kad_device_free(self.ctx.h, self.ptr)
        self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kad_mlp_create(ctx, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    out = _vp()
    _check(lib().kad_mlp_create(ctx, _p(p), C.byref(out)))
    return out


def kad_mlp_free(m):
    lib().kad_mlp_free(m)


def kad_mlp_get_params(m) -> np.ndarray:
    p = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(lib().kad_mlp_get_params(m, _p(p)))
    return p


def kad_mlp_loss_grad(m, d_x: int, d_y: int, rows: int):
    loss = C.c_float()
    grad = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(lib().kad_mlp_loss_grad(m, C.c_void_p(d_x), C.c_void_p(d_y), rows, C.byref(loss), _p(grad)))
    return loss.value, grad


def kad_mlp_train_step(m, d_x: int, d_y: int, rows: int, lr: float) -> float:
    loss = C.c_float()
    _check(lib().kad_mlp_train_step(m, C.c_void_p(d_x), C.c_void_p(d_y), rows, lr, C.byref(loss)))
    return loss.value


def kad_mlp_forward(m, d_x: int, rows: int) -> np.ndarray:
    y = np.zeros(rows, dtype=np.float32)
    _check(lib().kad_mlp_forward(m, C.c_void_p(d_x), rows, None, _p(y)))
    return y


def kad_mlp_train(ctx, graphs, btildes, omegas, epochs: int, batch: int, lr: float, lr_halve_every: int,
                  seed: int):
    """graphs: kad_graph handles; btildes: float64 arrays (caller numbering);
    omegas: one omega per graph.  Returns (params, norm, per-epoch losses)."""
    k = len(graphs)
    gs = (_vp * k)(*[g.value if hasattr(g, "value") else g for g in graphs])
    bts = [np.ascontiguousarray(b, dtype=np.float64) for b in btildes]
    bps = (_vp * k)(*[b.ctypes.data for b in bts])
    om = np.ascontiguousarray(omegas, dtype=np.float64)
    o = kad_train_opts(epochs, batch, lr, lr_halve_every, seed)
    params = np.zeros(MLP_PARAMS, dtype=np.float32)
    norm = np.zeros(6, dtype=np.float32)
    losses = np.zeros(epochs, dtype=np.float32)
    _check(lib().kad_mlp_train(ctx, gs, bps, _p(om), k, C.byref(o), _p(params), _p(norm), _p(losses)))
    return params, norm, losses


# ---------------------------------------------------------- convenience
# Handle owners.  A context frees what was made with it (samplers first,
# then graphs and MLPs) before itself; live contexts are closed at exit,
# before the HIP runtime is torn down.

_live_contexts = weakref.WeakSet()


@atexit.register
def _close_all():
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """Owns a kad_ctx (and optionally borrows a torch stream)."""

    def __init__(self, device: int = 0, hip_stream: int | None = None):
        self.h = kad_create(device, hip_stream)
        self._children = []          # weak references, in creation order
        _live_contexts.add(self)

    def _adopt(self, obj):
        self._children.append(weakref.ref(obj))

    def close(self):
        if self.h:
            kids = [r() for r in self._children]
            for rank in (0, 1):       # samplers / MLPs first, then graphs
                for k in kids:
                    if k is not None and (isinstance(k, Graph) == bool(rank)):
                        k.close()
            kad_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    def __init__(self, ctx: Context, g, validate: bool = False):
        self.ctx = ctx
        self.n = int(g.n)
        self.h = kad_graph_upload(ctx.h, g.row_ptr, g.col_idx, validate)
        ctx._adopt(self)

    def close(self):
        if self.h:
            kad_graph_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sampler:
    def __init__(self, graph: Graph, **opts):
        self.graph = graph
        self.n = graph.n
        self.opts = make_opts(**opts)
        self.h = kad_sampler_init(graph.ctx.h, graph.h, self.opts)
        graph.ctx._adopt(self)

    def close(self):
        if self.h:
            kad_sampler_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, seed: int):
        kad_sampler_reset(self.h, seed)

    def set_delta(self, dl, du):
        kad_set_delta(self.h, dl, du)

    def set_mlp_weights(self, params, norm):
        kad_set_mlp_weights(self.h, params, norm)

    def step_epoch(self) -> bool:
        return kad_step_epoch(self.h)

    def run_to_stop(self) -> kad_result:
        return kad_run_to_stop(self.h)

    def counts(self):
        return kad_fetch_counts(self.h, self.n)

    def btilde(self):
        return kad_fetch_btilde(self.h, self.n)

    def fg(self):
        return kad_fetch_fg(self.h, self.n)

    def delta_logs(self):
        return kad_fetch_delta(self.h, self.n)

    def result(self):
        return kad_fetch_result(self.h)

    def history(self, epochs: int):
        return kad_fetch_history(self.h, epochs)

    def calibration(self):
        return kad_fetch_calibration(self.h, self.n)

    def count_samples(self, stream, first, count):
        return kad_count_samples(self.h, stream, first, count, self.n)

    def sample_paths(self, stream, first, count, max_len):
        return kad_sample_paths(self.h, stream, first, count, max_len)
