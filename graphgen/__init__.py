"""Seeded synthetic graph inputs shared by the CPU oracle and the HIP path.

This module builds inputs only; it holds none of the sampling method's
arithmetic.  Every graph is undirected and unweighted (Sec. III), handed
over as a CSR with ascending neighbour ids, no self loops and no duplicate
edges, restricted to its largest connected component (Sec. V-A keeps only
the largest component of every instance).

Generators (all seeded; the stream of the generator's Philox key is 3):

* ``gnm``          -- Erdos-Renyi G(n, m): m distinct unordered pairs drawn
                      uniformly without replacement.
* ``rmat``         -- R-MAT with the Graph500 parameters (a,b,c,d) =
                      (0.57, 0.19, 0.19, 0.05), the paper's synthetic model
                      (Sec. V-A), 2^scale * edge_factor edge draws.
* ``road_grid``    -- a side x side 4-neighbour grid with a fraction of its
                      edges removed and a few short local shortcuts: a
                      stand-in for the paper's high-diameter road networks
                      (Table I).
* small closed-form families (path, star, cycle, complete, grid, hypercube)
  used by the tests.

Before the largest component is extracted the vertex ids are permuted by a
seeded random permutation, so that vertex ids carry no structure.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass

import numpy as np

GEN_STREAM = 3


@dataclass
class CSRGraph:
    """Undirected CSR: ``row_ptr`` int64[n+1], ``col_idx`` int32[nnz]."""

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), GEN_STREAM]))


def from_edges(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> CSRGraph:
    """Symmetrise, drop self loops and duplicates, sort adjacency."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSRGraph(n, row_ptr, dst.astype(np.int32), name)


def relabel_and_lcc(n: int, u: np.ndarray, v: np.ndarray, seed: int, name: str = "") -> CSRGraph:
    """Permute ids with a seeded permutation, then keep the largest component.

    Component ids are relabelled to 0..n'-1 in ascending order of the
    permuted id.
    """
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    perm = _rng(seed ^ 0x5EED).permutation(n).astype(np.int64)
    u = perm[np.asarray(u, dtype=np.int64)]
    v = perm[np.asarray(v, dtype=np.int64)]
    keep = u != v
    u, v = u[keep], v[keep]
    a = coo_matrix((np.ones(len(u), dtype=np.int8), (u, v)), shape=(n, n))
    ncomp, lab = connected_components(a, directed=False)
    if ncomp > 1:
        big = np.argmax(np.bincount(lab))
        inside = lab == big
    else:
        inside = np.ones(n, dtype=bool)
    newid = np.full(n, -1, dtype=np.int64)
    newid[inside] = np.arange(int(inside.sum()), dtype=np.int64)
    eu = newid[u]
    ev = newid[v]
    ok = (eu >= 0) & (ev >= 0)
    return from_edges(int(inside.sum()), eu[ok], ev[ok], name)


# ---------------------------------------------------------------- families


def gnm(n: int, m: int, seed: int) -> CSRGraph:
    """Erdos-Renyi G(n, m), restricted to its largest component."""
    rng = _rng(seed)
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("m exceeds the number of pairs")
    chosen = np.empty(0, dtype=np.int64)
    while len(chosen) < m:
        need = m - len(chosen)
        a = rng.integers(0, n, size=2 * need + 64, dtype=np.int64)
        b = rng.integers(0, n, size=2 * need + 64, dtype=np.int64)
        keep = a != b
        lo = np.minimum(a[keep], b[keep])
        hi = np.maximum(a[keep], b[keep])
        key = np.concatenate([chosen, lo * n + hi])
        _, first = np.unique(key, return_index=True)
        chosen = key[np.sort(first)]
    chosen = chosen[:m]
    return relabel_and_lcc(n, chosen // n, chosen % n, seed, f"gnm_{n}_{m}_s{seed}")


def rmat_edges(scale: int, edge_factor: int, seed: int,
               abcd=(0.57, 0.19, 0.19, 0.05), chunk: int = 1 << 24):
    """Raw R-MAT edge draws (2^scale * edge_factor of them)."""
    a, b, c, _ = abcd
    rng = _rng(seed)
    total = (1 << scale) * edge_factor
    us, vs = [], []
    done = 0
    while done < total:
        cnt = min(chunk, total - done)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(cnt)
            ubit = r >= a + b                    # quadrants c, d: row bit set
            vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)   # b, d
            u = (u << 1) | ubit
            v = (v << 1) | vbit
        us.append(u)
        vs.append(v)
        done += cnt
    return np.concatenate(us), np.concatenate(vs)


def rmat_numpy(scale: int, edge_factor: int, seed: int) -> CSRGraph:
    """R-MAT (Graph500 a,b,c,d), symmetrised, deduplicated, largest component."""
    u, v = rmat_edges(scale, edge_factor, seed)
    return relabel_and_lcc(1 << scale, u, v, seed, f"rmat_{scale}_{edge_factor}_s{seed}")


_HERE = os.path.dirname(os.path.abspath(__file__))
_NATIVE = os.path.join(_HERE, "librmatgen.so")


def build_native(force: bool = True) -> str:
    """Compile rmatgen.c (the threaded R-MAT builder) with gcc."""
    import subprocess
    if force or not os.path.exists(_NATIVE):
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
                               "-pthread", "-shared", "-fPIC", "-o", _NATIVE,
                               os.path.join(_HERE, "rmatgen.c"), "-lm"])
    return _NATIVE


def _native_lib():
    import ctypes
    if not os.path.exists(_NATIVE):
        return None
    lib = ctypes.CDLL(_NATIVE)
    lib.kg_rmat.restype = ctypes.c_void_p
    lib.kg_rmat.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                            ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_int]
    lib.kg_hyperbolic.restype = ctypes.c_void_p
    lib.kg_hyperbolic.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.kg_n.restype = ctypes.c_int32
    lib.kg_n.argtypes = [ctypes.c_void_p]
    lib.kg_nnz.restype = ctypes.c_int64
    lib.kg_nnz.argtypes = [ctypes.c_void_p]
    lib.kg_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.kg_free.argtypes = [ctypes.c_void_p]
    return lib


def rmat_native(scale: int, edge_factor: int, seed: int, threads: int = 0) -> CSRGraph:
    """The same graph as rmat_numpy, built by the threaded C builder."""
    lib = _native_lib()
    if lib is None:
        raise RuntimeError("librmatgen.so is not built (graphgen.build_native())")
    n = 1 << scale
    perm = np.ascontiguousarray(_rng(seed ^ 0x5EED).permutation(n).astype(np.int64))
    if threads <= 0:
        threads = max(1, min(16, os.cpu_count() or 1))
    h = lib.kg_rmat(scale, edge_factor, seed & (2**64 - 1), GEN_STREAM, 0.57, 0.19, 0.19,
                    perm.ctypes.data, threads)
    if not h:
        raise MemoryError("R-MAT builder failed")
    try:
        nn = lib.kg_n(h)
        nnz = lib.kg_nnz(h)
        rp = np.empty(nn + 1, dtype=np.int64)
        ci = np.empty(nnz, dtype=np.int32)
        lib.kg_copy(h, rp.ctypes.data, ci.ctypes.data)
    finally:
        lib.kg_free(h)
    return CSRGraph(nn, rp, ci, f"rmat_{scale}_{edge_factor}_s{seed}")


def hyperbolic(scale: int, avg_deg: float, seed: int, gamma: float = 3.0, threads: int = 0) -> CSRGraph:
    """Random hyperbolic graph (threshold model) with 2^scale points, power-law
    degree exponent gamma, expected average degree avg_deg (|E| = avg_deg/2
    |V|), seeded relabelling, largest component (the threaded C builder)."""
    import ctypes
    lib = _native_lib()
    if lib is None:
        raise RuntimeError("librmatgen.so is not built (graphgen.build_native())")
    n = 1 << scale
    perm = np.ascontiguousarray(_rng(seed ^ 0x5EED).permutation(n).astype(np.int64))
    if threads <= 0:
        threads = max(1, min(16, os.cpu_count() or 1))
    R = ctypes.c_double()
    h = lib.kg_hyperbolic(scale, float(avg_deg), float(gamma), seed & (2**64 - 1), GEN_STREAM, perm.ctypes.data,
                          threads, ctypes.byref(R))
    if not h:
        raise MemoryError("hyperbolic builder failed")
    try:
        nn = lib.kg_n(h)
        nnz = lib.kg_nnz(h)
        rp = np.empty(nn + 1, dtype=np.int64)
        ci = np.empty(nnz, dtype=np.int32)
        lib.kg_copy(h, rp.ctypes.data, ci.ctypes.data)
    finally:
        lib.kg_free(h)
    return CSRGraph(nn, rp, ci, f"hyp_{scale}_{avg_deg:g}_g{gamma:g}_s{seed}")


def rmat(scale: int, edge_factor: int, seed: int) -> CSRGraph:
    """R-MAT (Graph500 a,b,c,d), symmetrised, deduplicated, largest component
    (the threaded builder when it is built, else numpy; both give the same
    graph)."""
    if _native_lib() is not None:
        return rmat_native(scale, edge_factor, seed)
    return rmat_numpy(scale, edge_factor, seed)


def road_grid(side: int, seed: int, p_drop: float = 0.05, shortcut_frac: float = 0.001,
              max_off: int = 8) -> CSRGraph:
    """Perturbed 2-D grid: drop each edge with prob. p_drop, add local shortcuts."""
    rng = _rng(seed)
    ids = np.arange(side * side, dtype=np.int64).reshape(side, side)
    hu = ids[:, :-1].ravel()
    hv = ids[:, 1:].ravel()
    vu = ids[:-1, :].ravel()
    vv = ids[1:, :].ravel()
    u = np.concatenate([hu, vu])
    v = np.concatenate([hv, vv])
    keep = rng.random(len(u)) >= p_drop
    u, v = u[keep], v[keep]
    k = int(np.ceil(shortcut_frac * len(u)))
    su = np.empty(0, dtype=np.int64)
    sv = np.empty(0, dtype=np.int64)
    while len(su) < k:
        cnt = 2 * (k - len(su)) + 16
        base = rng.integers(0, side * side, size=cnt, dtype=np.int64)
        dx = rng.integers(-max_off, max_off + 1, size=cnt, dtype=np.int64)
        dy = rng.integers(-max_off, max_off + 1, size=cnt, dtype=np.int64)
        x = np.clip(base % side + dx, 0, side - 1)
        y = np.clip(base // side + dy, 0, side - 1)
        tgt = y * side + x
        ok = tgt != base
        su = np.concatenate([su, base[ok]])
        sv = np.concatenate([sv, tgt[ok]])
    u = np.concatenate([u, su[:k]])
    v = np.concatenate([v, sv[:k]])
    return relabel_and_lcc(side * side, u, v, seed, f"grid_{side}_s{seed}")


# ------------------------------------------------- small closed-form graphs


def path_graph(n: int) -> CSRGraph:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, f"path_{n}")


def star_graph(n: int) -> CSRGraph:
    """Centre 0 with n-1 leaves."""
    i = np.arange(1, n)
    return from_edges(n, np.zeros(n - 1, dtype=np.int64), i, f"star_{n}")


def cycle_graph(n: int) -> CSRGraph:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, f"cycle_{n}")


def complete_graph(n: int) -> CSRGraph:
    a, b = np.triu_indices(n, 1)
    return from_edges(n, a, b, f"complete_{n}")


def grid_graph(rows: int, cols: int) -> CSRGraph:
    """Unperturbed grid, vertex id = r * cols + c."""
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_edges(rows * cols, u, v, f"grid_{rows}x{cols}")


def hypercube_graph(k: int) -> CSRGraph:
    n = 1 << k
    u, v = [], []
    for x in range(n):
        for b in range(k):
            y = x ^ (1 << b)
            if x < y:
                u.append(x)
                v.append(y)
    return from_edges(n, np.array(u), np.array(v), f"hypercube_{k}")


def random_connected(n: int, extra: int, seed: int) -> CSRGraph:
    """Random spanning tree plus ``extra`` random edges (no relabelling)."""
    rng = _rng(seed)
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    u = list(range(1, n))
    v = list(parent)
    if extra:
        a = rng.integers(0, n, size=extra)
        b = rng.integers(0, n, size=extra)
        u += list(a)
        v += list(b)
    return from_edges(n, np.array(u), np.array(v), f"rc_{n}_{extra}_s{seed}")


# ------------------------------------------------------------- workloads

WORKLOADS = {
    # name: (builder, kwargs, description)
    "er2048": (gnm, dict(n=2048, m=16384, seed=1),
               "Erdos-Renyi G(2048, 16384), largest component"),
    "rmat20": (rmat, dict(scale=20, edge_factor=16, seed=2),
               "R-MAT scale 20, edge factor 16, Graph500 parameters"),
    "grid2048": (road_grid, dict(side=2048, seed=3),
                 "2048x2048 grid, 5% edges removed, 0.1% shortcuts of offset <= 8"),
    "rmat22": (rmat, dict(scale=22, edge_factor=16, seed=1022),
               "R-MAT scale 22, edge factor 16 (held-out graph for the learned prior)"),
    "rmat26": (rmat, dict(scale=26, edge_factor=16, seed=26),
               "R-MAT scale 26, edge factor 16 (about 1e9 undirected edges)"),
}
# the graph-size sweep: R-MAT and random hyperbolic graphs (power-law
# exponent 3) with |E| = 30 |V| at 2^23 .. 2^25 vertices; at 2^26 the
# adjacency would pass 2^31 entries, so R-MAT takes edge factor 16 (the
# large configuration above) and the hyperbolic graph |E| = 15 |V|
for _s in (23, 24, 25):
    WORKLOADS[f"rmat{_s}_ef30"] = (rmat, dict(scale=_s, edge_factor=30, seed=_s),
                                   f"R-MAT scale {_s}, edge factor 30")
    WORKLOADS[f"hyp{_s}"] = (hyperbolic, dict(scale=_s, avg_deg=60.0, seed=_s),
                             f"random hyperbolic graph, 2^{_s} points, gamma 3, average degree 60")
WORKLOADS["hyp26"] = (hyperbolic, dict(scale=26, avg_deg=30.0, seed=26),
                      "random hyperbolic graph, 2^26 points, gamma 3, average degree 30")


def cache_dir() -> str:
    d = os.environ.get("KAD_GRAPH_CACHE", os.path.join("/tmp", "kadgraphs"))
    os.makedirs(d, exist_ok=True)
    return d


def cached(builder, **kw) -> CSRGraph:
    """Build a graph once and keep it as an .npz file keyed by its recipe."""
    key = builder.__name__ + "_" + "_".join(f"{k}{v}" for k, v in sorted(kw.items()))
    h = hashlib.sha1(key.encode()).hexdigest()[:10]
    path = os.path.join(cache_dir(), f"{key}_{h}.npz")
    if os.path.exists(path):
        z = np.load(path)
        return CSRGraph(int(z["n"]), z["row_ptr"], z["col_idx"], str(z["name"]))
    g = builder(**kw)
    tmp = path + f".tmp{os.getpid()}.npz"
    np.savez(tmp, n=g.n, row_ptr=g.row_ptr, col_idx=g.col_idx, name=g.name)
    os.replace(tmp, path)
    return g


def workload(name: str) -> CSRGraph:
    builder, kw, _ = WORKLOADS[name]
    return cached(builder, **kw)


def training_graphs(count: int = 20, first_seed: int = 101):
    """Training set for the learned prior: R-MAT scales 16, 17, 18 cycling."""
    return [cached(rmat, scale=16 + (i % 3), edge_factor=16, seed=first_seed + i)
            for i in range(count)]
