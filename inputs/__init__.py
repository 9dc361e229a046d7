"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Holds no BFS or codec arithmetic: only graphs (R-MAT / uniform CSR), BFS
roots, destination-segment bounds, MLP initial weights and random sorted
ID sets, all as plain numpy arrays.  The native part is ``gen.c`` (built with
gcc + OpenMP into ``libbfsgen.so`` next to this file).

Workload recipe (the paper's Graph 500 setting, "Synthetic data" section):
``V = 2^scale`` vertices, ``edgefactor * V`` edge samples, R-MAT quadrant
probabilities (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), undirected, self-loops
and duplicates removed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libbfsgen.so")
_lock = threading.Lock()
_lib = None

RMAT = 0
UNIFORM = 1
RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = False) -> str:
    """Compile gen.c into libbfsgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            u64, u32, i32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
            vp = ctypes.c_void_p
            lib.bfsgen_mix64.restype = u64
            lib.bfsgen_mix64.argtypes = [u64]
            lib.bfsgen_ctr.restype = u64
            lib.bfsgen_ctr.argtypes = [u64, u64, u64]
            lib.bfsgen_graph_create.restype = vp
            lib.bfsgen_graph_create.argtypes = [i32, i32, i32, u64, dbl, dbl, dbl]
            lib.bfsgen_graph_info.restype = None
            lib.bfsgen_graph_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u64),
                                              ctypes.POINTER(ctypes.POINTER(u64)),
                                              ctypes.POINTER(ctypes.POINTER(u32))]
            lib.bfsgen_graph_free.restype = None
            lib.bfsgen_graph_free.argtypes = [vp]
            lib.bfsgen_samples.restype = None
            lib.bfsgen_samples.argtypes = [i32, i32, u64, dbl, dbl, dbl, u64, u64, vp, vp]
            lib.bfsgen_roots.restype = i32
            lib.bfsgen_roots.argtypes = [vp, i32, u64, i32, vp]
            lib.bfsgen_bounds_equal.restype = None
            lib.bfsgen_bounds_equal.argtypes = [u64, u32, vp]
            lib.bfsgen_bounds_zipf.restype = i32
            lib.bfsgen_bounds_zipf.argtypes = [u64, u32, dbl, u32, u64, vp, vp]
            lib.bfsgen_zipf_draws.restype = None
            lib.bfsgen_zipf_draws.argtypes = [dbl, u32, u64, u64, vp]
            lib.bfsgen_uniform_f32.restype = None
            lib.bfsgen_uniform_f32.argtypes = [u64, u64, u64, ctypes.c_float, vp]
            _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class Graph:
    """Symmetric CSR graph: ``row_ptr`` u64[V+1], ``col_idx`` u32[arcs], rows ascending."""

    def __init__(self, kind: int, scale: int, edgefactor: int, seed: int):
        lib = _load()
        a, b, c = RMAT_ABC
        h = lib.bfsgen_graph_create(kind, scale, edgefactor, seed, a, b, c)
        if not h:
            raise MemoryError("graph generation failed (scale=%d)" % scale)
        self._h = h
        # kept for __del__: module globals may already be gone at interpreter exit
        self._free = lib.bfsgen_graph_free
        nv, na = ctypes.c_uint32(), ctypes.c_uint64()
        rp, ci = ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)()
        lib.bfsgen_graph_info(h, ctypes.byref(nv), ctypes.byref(na), ctypes.byref(rp), ctypes.byref(ci))
        self.kind, self.scale, self.edgefactor, self.seed = kind, scale, edgefactor, seed
        self.n_vertices = int(nv.value)
        self.n_arcs = int(na.value)
        self.row_ptr = np.ctypeslib.as_array(rp, shape=(self.n_vertices + 1,))
        self.col_idx = (np.ctypeslib.as_array(ci, shape=(self.n_arcs,)) if self.n_arcs
                        else np.zeros(0, np.uint32))

    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            self.row_ptr = None
            self.col_idx = None
            self._free(h)

    @property
    def name(self) -> str:
        return "%s-s%d-ef%d-seed%d" % ("rmat" if self.kind == RMAT else "uniform",
                                       self.scale, self.edgefactor, self.seed)


_graph_cache: dict = {}


def graph(kind: int = RMAT, scale: int = 16, edgefactor: int = 16, seed: int = 1,
          cache: bool = True) -> Graph:
    key = (kind, scale, edgefactor, seed)
    if cache and key in _graph_cache:
        return _graph_cache[key]
    g = Graph(kind, scale, edgefactor, seed)
    if cache:
        _graph_cache[key] = g
    return g


def clear_cache() -> None:
    _graph_cache.clear()


def samples(kind: int, scale: int, seed: int, first: int, count: int):
    """Raw edge samples (u, v) before symmetrisation, for statistics tests."""
    lib = _load()
    u = np.empty(count, np.uint32)
    v = np.empty(count, np.uint32)
    a, b, c = RMAT_ABC
    lib.bfsgen_samples(kind, scale, seed, a, b, c, first, count, _ptr(u), _ptr(v))
    return u, v


def roots(g: Graph, k: int, seed: int = 1) -> np.ndarray:
    """k distinct seeded roots with positive degree."""
    out = np.empty(k, np.uint32)
    n = _load().bfsgen_roots(_ptr(g.row_ptr), g.scale, seed, k, _ptr(out))
    return out[:n]


def bounds_equal(n_vertices: int, nseg: int) -> np.ndarray:
    out = np.empty(nseg + 1, np.uint32)
    _load().bfsgen_bounds_equal(n_vertices, nseg, _ptr(out))
    return out


def bounds_zipf(n_vertices: int, nseg: int, seed: int = 1, s: float = 1.2,
                kmax: int = 1 << 20):
    """Zipf(s)-sized contiguous ranges tiling [0, V): (bounds u32[R+1], draws u32[R])."""
    out = np.empty(nseg + 1, np.uint32)
    ks = np.empty(nseg, np.uint32)
    rc = _load().bfsgen_bounds_zipf(n_vertices, nseg, s, kmax, seed, _ptr(out), _ptr(ks))
    if rc != 0:
        raise MemoryError("zipf table")
    return out, ks


def zipf_draws(count: int, seed: int = 1, s: float = 1.2, kmax: int = 1 << 20) -> np.ndarray:
    out = np.empty(count, np.uint32)
    _load().bfsgen_zipf_draws(s, kmax, seed, count, _ptr(out))
    return out


def ctr(seed: int, stream: int, idx: int) -> int:
    return int(_load().bfsgen_ctr(seed, stream, idx))


def mix64(z: int) -> int:
    return int(_load().bfsgen_mix64(z))


MLP_SHAPE = (8, 64, 64, 35)


def mlp_init(seed: int = 1) -> np.ndarray:
    """He-uniform initial weights, flat fp32 in the order W1 b1 W2 b2 W3 b3
    (row-major [out][in]); biases zero.  Stream 100+layer of the counter RNG."""
    parts = []
    dims = MLP_SHAPE
    for layer in range(3):
        fan_in, fan_out = dims[layer], dims[layer + 1]
        lim = np.float32(np.sqrt(6.0 / fan_in))
        w = np.empty(fan_out * fan_in, np.float32)
        _load().bfsgen_uniform_f32(seed, 100 + layer, w.size, lim, _ptr(w))
        parts.append(w)
        parts.append(np.zeros(fan_out, np.float32))
    return np.concatenate(parts)


def mlp_param_count() -> int:
    d = MLP_SHAPE
    return sum(d[i] * d[i + 1] + d[i + 1] for i in range(3))


def random_sorted(n: int, universe: int, seed: int, lo: int = 0) -> np.ndarray:
    """n distinct uint32 values in [lo, lo+universe), ascending."""
    rng = np.random.default_rng(seed)
    if n > universe:
        raise ValueError("n > universe")
    if universe <= 4 * n or universe <= (1 << 22):
        vals = rng.choice(universe, size=n, replace=False)
    else:
        vals = np.unique(rng.integers(0, universe, size=int(n * 1.2) + 16, dtype=np.int64))
        while vals.size < n:
            vals = np.unique(np.concatenate([vals, rng.integers(0, universe, size=n, dtype=np.int64)]))
        vals = rng.choice(vals, size=n, replace=False)
    return np.sort(vals.astype(np.int64) + lo).astype(np.uint32)


def clustered_sorted(n: int, universe: int, seed: int, lo: int = 0, runs: int = 8) -> np.ndarray:
    """Sorted distinct values made of dense runs separated by large gaps:
    exercises bitmap, small-width and exception-carrying blocks."""
    rng = np.random.default_rng(seed)
    out = set()
    while len(out) < n:
        start = int(rng.integers(0, max(1, universe - 4096)))
        width = int(rng.integers(1, 4096))
        dens = float(rng.uniform(0.05, 1.0))
        k = min(n - len(out), max(1, int(width * dens)))
        pts = rng.choice(width, size=min(k, width), replace=False) + start
        out.update(int(x) for x in pts if x < universe)
    arr = np.array(sorted(out)[:n], dtype=np.int64) + lo
    return arr.astype(np.uint32)
