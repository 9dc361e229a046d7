"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow reference implementations of every step of the frontier-codec
path: a textbook FIFO BFS and its invariant checker, the frontier
partitioner, the scalar block codec (writer and validating reader), the
codec selectors, the selector features, the resolve rules (``oracle.c``,
plain C built with gcc), the MLP in fp64 numpy (``mlp.py``), and the
candidate exchange of the compressed 2D BFS (unfiltered candidates per owner,
the receiver's merge and visited filter; numpy below).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "bitmap.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

ST_OK, ST_INVAL, ST_CAPACITY, ST_CORRUPT = 0, 1, 2, 3
PLAIN_BP, EXHAUSTIVE = 0, 1
CLS_BITMAP, CLS_PFOR = 0, 34
BLOCK = 128
GROUP = 16
# Compression threshold: segments of fewer IDs are sent raw (the "Usage of
# compression thresholds" section).  The value is this project's reading:
# on the R-MAT and uniform frontiers measured, the compressed form is never
# smaller than raw below about 15 IDs, and below about 33 at the widest gaps a
# scale-26 segment can have.
RAW_BELOW = 32


def build(force: bool = False) -> str:
    """Compile oracle.c and bitmap.c (plain C, no fast-math) into liboracle.so."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
            sig = {
                "ref_bfs": (ctypes.c_int32, [u32, vp, vp, u32, vp, vp]),
                "ref_bfs_check": (i32, [u32, vp, vp, u32, vp, vp]),
                "ref_frontier": (u64, [u32, vp, ctypes.c_int32, vp]),
                "ref_partition": (None, [vp, u64, vp, u32, vp]),
                "ref_bitlen": (u32, [u64]),
                "ref_encode_bound": (u64, [u64, u32]),
                "ref_select": (i32, [vp, vp, vp, vp, u32, i32, vp]),
                "ref_block_details": (i32, [vp, vp, u32, vp, vp, vp, vp, vp, vp]),
                "ref_encode": (i32, [vp, vp, vp, vp, u32, vp, i32, u32, vp, u64, vp]),
                "ref_encoded_size": (u64, [vp, vp, u32, vp, i32, u32]),
                "ref_decode": (i32, [vp, vp, u32, vp, u64, vp]),
                "ref_f32_to_f16": (ctypes.c_uint16, [ctypes.c_float]),
                "ref_features": (i32, [vp, vp, u32, vp, vp]),
                "ref_resolve": (u64, [vp, vp, u32, vp, i32, vp]),
                "ref_bmc_bound": (u64, [u64, u32]),
                "ref_bmc_classes": (u64, [vp, vp, u32, vp]),
                "ref_bmc_encode": (i32, [vp, vp, u32, vp, u64, vp]),
                "ref_bmc_decode": (i32, [vp, vp, u32, vp, u64, vp]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


# ---------------------------------------------------------------- BFS

def bfs(g, root: int):
    """Textbook FIFO BFS -> (level i32[V], parent i32[V], depth)."""
    V = g.n_vertices
    level = np.empty(V, np.int32)
    parent = np.empty(V, np.int32)
    depth = _load().ref_bfs(V, _p(g.row_ptr), _p(g.col_idx), int(root), _p(level), _p(parent))
    if depth < 0:
        raise MemoryError("oracle BFS queue")
    return level, parent, int(depth)


def bfs_check(g, root: int, level: np.ndarray, parent: np.ndarray) -> int:
    level = np.ascontiguousarray(level, np.int32)
    parent = np.ascontiguousarray(parent, np.int32)
    return int(_load().ref_bfs_check(g.n_vertices, _p(g.row_ptr), _p(g.col_idx), int(root),
                                     _p(level), _p(parent)))


def frontier(level: np.ndarray, L: int) -> np.ndarray:
    level = np.ascontiguousarray(level, np.int32)
    out = np.empty(level.size, np.uint32)
    k = _load().ref_frontier(level.size, _p(level), int(L), _p(out))
    return out[:k].copy()


def frontiers(level: np.ndarray, depth: int):
    return [frontier(level, L) for L in range(depth + 1)]


def partition(ids: np.ndarray, bounds: np.ndarray) -> np.ndarray:
    ids, bounds = _u32(ids), _u32(bounds)
    nseg = bounds.size - 1
    seg_off = np.empty(nseg + 1, np.uint64)
    _load().ref_partition(_p(ids), ids.size, _p(bounds), nseg, _p(seg_off))
    return seg_off


# ---------------------------------------------------------------- codec

class Batch:
    """A batch of segments: ids u32[n] (concatenated), seg_off u64[R+1],
    seg_lo/seg_hi u32[R] (each segment's ID range), seg_level i32[R]."""

    def __init__(self, ids, seg_off, seg_lo, seg_hi, seg_level=None):
        self.ids = _u32(ids)
        self.seg_off = _u64(seg_off)
        self.seg_lo = _u32(seg_lo)
        self.seg_hi = _u32(seg_hi)
        self.nseg = self.seg_lo.size
        self.seg_level = (np.zeros(self.nseg, np.int32) if seg_level is None
                          else np.ascontiguousarray(seg_level, np.int32))
        assert self.seg_off.size == self.nseg + 1 and self.seg_hi.size == self.nseg

    @property
    def n_ids(self) -> int:
        return int(self.ids.size)

    @property
    def n_blocks(self) -> int:
        n = np.diff(self.seg_off.astype(np.int64))
        return int(((n + BLOCK - 1) // BLOCK).sum())


def batch_from_frontier(ids, bounds, level: int = 0) -> Batch:
    """One frontier split by vertex-ID range into len(bounds)-1 segments."""
    bounds = _u32(bounds)
    seg_off = partition(ids, bounds)
    R = bounds.size - 1
    return Batch(ids, seg_off, bounds[:-1], bounds[1:], np.full(R, level, np.int32))


def concat_batches(batches) -> Batch:
    ids, offs, lo, hi, lev = [], [np.zeros(1, np.uint64)], [], [], []
    base = 0
    for b in batches:
        ids.append(b.ids)
        offs.append(b.seg_off[1:] + np.uint64(base))
        base += b.n_ids
        lo.append(b.seg_lo)
        hi.append(b.seg_hi)
        lev.append(b.seg_level)
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return Batch(cat(ids, np.uint32), np.concatenate(offs), cat(lo, np.uint32), cat(hi, np.uint32),
                 cat(lev, np.int32))


def encode_bound(n_ids: int, nseg: int) -> int:
    return int(_load().ref_encode_bound(n_ids, nseg))


def select(b: Batch, mode: int = EXHAUSTIVE) -> np.ndarray:
    cls = np.empty(max(1, b.n_blocks), np.uint8)
    st = _load().ref_select(_p(b.ids), _p(b.seg_off), _p(b.seg_lo), _p(b.seg_hi), b.nseg, mode,
                            _p(cls))
    if st != ST_OK:
        raise ValueError("oracle select: status %d" % st)
    return cls[:b.n_blocks].copy()


def block_details(b: Batch, classes=None):
    nb = b.n_blocks
    out = {k: np.zeros(max(1, nb), np.uint32) for k in ("words", "wmin", "span", "pfor_b", "pfor_e")}
    cls = None if classes is None else np.ascontiguousarray(classes, np.uint8)
    _load().ref_block_details(_p(b.ids), _p(b.seg_off), b.nseg, _p(cls), _p(out["words"]),
                              _p(out["wmin"]), _p(out["span"]), _p(out["pfor_b"]), _p(out["pfor_e"]))
    return {k: v[:nb] for k, v in out.items()}


def encode(b: Batch, classes=None, mode: int = EXHAUSTIVE, cap: int | None = None,
           raw_below: int = RAW_BELOW):
    """-> (stream u8[total], seg_byte_off u64[R+1]); raises on INVAL/CAPACITY.
    Segments of fewer than raw_below IDs are written raw, empty ones as no
    bytes."""
    st, buf, sbo = encode_status(b, classes, mode, cap, raw_below)
    if st != ST_OK:
        raise ValueError("oracle encode: status %d" % st)
    return buf, sbo


def encode_status(b: Batch, classes=None, mode: int = EXHAUSTIVE, cap: int | None = None,
                  raw_below: int = RAW_BELOW):
    if cap is None:
        cap = encode_bound(b.n_ids, b.nseg)
    buf = np.zeros(max(1, cap), np.uint8)
    sbo = np.zeros(b.nseg + 1, np.uint64)
    cls = None if classes is None else np.ascontiguousarray(classes, np.uint8)
    st = _load().ref_encode(_p(b.ids), _p(b.seg_off), _p(b.seg_lo), _p(b.seg_hi), b.nseg, _p(cls),
                            mode, int(raw_below), _p(buf), cap, _p(sbo))
    if st != ST_OK:
        return st, None, None
    return st, buf[:int(sbo[-1])].copy(), sbo


def encoded_size(b: Batch, classes=None, mode: int = EXHAUSTIVE, raw_below: int = RAW_BELOW) -> int:
    cls = None if classes is None else np.ascontiguousarray(classes, np.uint8)
    return int(_load().ref_encoded_size(_p(b.ids), _p(b.seg_off), b.nseg, _p(cls), mode,
                                        int(raw_below)))


def decode(stream: np.ndarray, seg_byte_off: np.ndarray, out_cap: int | None = None):
    """-> (status, ids u32[n], out_off u64[R+1])."""
    stream = np.ascontiguousarray(stream, np.uint8)
    if stream.size == 0:
        stream = np.zeros(4, np.uint8)
    sbo = _u64(seg_byte_off)
    nseg = sbo.size - 1
    if out_cap is None:
        # a segment of n IDs takes at least 4 n bytes (raw) or 16 + 8
        # ceil(n/128) bytes (compressed), so n <= 16 * bytes
        out_cap = 16 * (int(sbo[-1]) if nseg else 0) + 1
    out = np.zeros(max(1, out_cap), np.uint32)
    off = np.zeros(nseg + 1, np.uint64)
    st = _load().ref_decode(_p(stream), _p(sbo), nseg, _p(out), out_cap, _p(off))
    if st != ST_OK:
        return st, None, None
    return st, out[:int(off[-1])].copy(), off


def f32_to_f16(x: float) -> int:
    return int(_load().ref_f32_to_f16(float(x)))


def features(b: Batch) -> np.ndarray:
    """u16 fp16 bit patterns [n_blocks, 8]."""
    nb = b.n_blocks
    out = np.zeros((max(1, nb), 8), np.uint16)
    _load().ref_features(_p(b.ids), _p(b.seg_off), b.nseg, _p(b.seg_level), _p(out))
    return out[:nb].copy()


def resolve(b: Batch, pred: np.ndarray, literal: bool = False):
    """-> (resolved classes u8[nb], number of exhaustive fallbacks)."""
    pred = np.ascontiguousarray(pred, np.uint8)
    out = np.zeros(max(1, b.n_blocks), np.uint8)
    fb = _load().ref_resolve(_p(b.ids), _p(b.seg_off), b.nseg, _p(pred), int(literal), _p(out))
    return out[:b.n_blocks].copy(), int(fb)


def bitlen(x: int) -> int:
    return int(_load().ref_bitlen(int(x)))


def entropy(x: np.ndarray) -> float:
    """Empirical Shannon entropy, eq. (2): -sum p_i log2 p_i over distinct values."""
    x = np.asarray(x)
    if x.size == 0:
        return 0.0
    _, counts = np.unique(x, return_counts=True)
    p = counts / x.size
    return float(-(p * np.log2(p)).sum())


def gap_entropy(ids: np.ndarray) -> float:
    """Entropy of the gaps of a sorted ID list (the empirical bound reported
    per level, eq. (2)/(3))."""
    ids = np.asarray(ids, np.int64)
    return entropy(np.diff(ids)) if ids.size > 1 else 0.0


def ratio(raw_bytes: int, compressed_bytes: int) -> float:
    """Compression ratio, eq. (4): original size / compressed size."""
    return raw_bytes / compressed_bytes if compressed_bytes else float("inf")


def ratio_percent(raw_bytes: int, compressed_bytes: int) -> float:
    """Compression ratio in percent, eq. (10): 100 / ratio."""
    return 100.0 / ratio(raw_bytes, compressed_bytes)


# ---------------------------------------------------------------- candidate exchange

def candidates(g, frontier_ids, bounds, level: int = 0) -> Batch:
    """The row exchange of the compressed 2D BFS (the candidate vector t = A x f
    compressed and sent to its owners before the visited filter), on one
    address space.  Owner p holds the frontier vertices in [bounds[p],
    bounds[p+1]); its candidate set T_p is every neighbour of those vertices,
    visited or not, sorted and without repeats; segment p*R + d of the batch
    is T_p restricted to owner d's range [bounds[d], bounds[d+1]).  A vertex
    that several owners reach appears in each of their sets."""
    bounds = _u32(bounds)
    fr = _u32(frontier_ids)
    R = bounds.size - 1
    rp = np.asarray(g.row_ptr, np.int64)
    ids, offs, lo, hi = [], [np.zeros(1, np.uint64)], [], []
    base = 0
    for p in range(R):
        fp = fr[(fr >= bounds[p]) & (fr < bounds[p + 1])]
        if fp.size:
            nb = np.concatenate([g.col_idx[rp[u]:rp[u + 1]] for u in fp.tolist()])
        else:
            nb = np.zeros(0, np.uint32)
        tp = np.unique(nb.astype(np.uint32))
        off = partition(tp, bounds)
        ids.append(tp)
        offs.append(off[1:].astype(np.uint64) + np.uint64(base))
        base += tp.size
        lo.append(bounds[:-1])
        hi.append(bounds[1:])
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return Batch(cat(ids, np.uint32), np.concatenate(offs), cat(lo, np.uint32), cat(hi, np.uint32),
                 np.full(R * R, level, np.int32))


def merge_filter(ids, level: np.ndarray, cur_level: int):
    """The receiving side: the union of every received candidate, less the
    visited vertices (level >= 0), is the next frontier (sorted); those get
    level cur_level + 1.  Returns (frontier u32, new level array)."""
    u = np.unique(_u32(ids))
    lv = np.ascontiguousarray(level, np.int32).copy()
    new = u[lv[u] < 0]
    lv[new] = cur_level + 1
    return new.astype(np.uint32), lv


# ---------------------------------------------------------------- bitmap codec

BMC_ZERO, BMC_ONES, BMC_SET, BMC_CLEAR, BMC_LITERAL = 0, 1, 2, 3, 4
BMC_BLOCK_WORDS = 128


def bmc_bound(n_words: int, nseg: int) -> int:
    return int(_load().ref_bmc_bound(int(n_words), int(nseg)))


def bmc_encode(bits: np.ndarray, seg_w: np.ndarray):
    """Bitmap codec: words bits u32, segments seg_w u64[R+1] (word ranges)
    -> (stream u8, seg_byte_off u64[R+1])."""
    bits, seg_w = _u32(bits), _u64(seg_w)
    if bits.size == 0:
        bits = np.zeros(1, np.uint32)
    nseg = seg_w.size - 1
    cap = bmc_bound(int(seg_w[-1] - seg_w[0]) if nseg else 0, nseg)
    out = np.zeros(max(4, cap), np.uint8)
    sbo = np.zeros(nseg + 1, np.uint64)
    st = _load().ref_bmc_encode(_p(bits), _p(seg_w), nseg, _p(out), cap, _p(sbo))
    if st != ST_OK:
        raise ValueError("bitmap encode status %d" % st)
    return out[:int(sbo[-1])].copy(), sbo


def bmc_classes(bits: np.ndarray, seg_w: np.ndarray) -> np.ndarray:
    bits, seg_w = _u32(bits), _u64(seg_w)
    if bits.size == 0:
        bits = np.zeros(1, np.uint32)
    nseg = seg_w.size - 1
    nblk = int(sum((int(seg_w[r + 1] - seg_w[r]) + BMC_BLOCK_WORDS - 1) // BMC_BLOCK_WORDS
                   for r in range(nseg)))
    cls = np.zeros(max(1, nblk), np.uint8)
    k = _load().ref_bmc_classes(_p(bits), _p(seg_w), nseg, _p(cls))
    return cls[:k]


def bmc_decode(stream: np.ndarray, seg_byte_off: np.ndarray, out_cap: int | None = None):
    """-> (status, words u32[n], out_off u64[R+1])."""
    stream = np.ascontiguousarray(stream, np.uint8)
    if stream.size == 0:
        stream = np.zeros(4, np.uint8)
    sbo = _u64(seg_byte_off)
    nseg = sbo.size - 1
    if out_cap is None:
        # a segment of nw words takes at least 16 + 12 ceil(nw / 128) bytes
        out_cap = 11 * (int(sbo[-1]) if nseg else 0) + 1
    out = np.zeros(max(1, out_cap), np.uint32)
    off = np.zeros(nseg + 1, np.uint64)
    st = _load().ref_bmc_decode(_p(stream), _p(sbo), nseg, _p(out), out_cap, _p(off))
    if st != ST_OK:
        return st, None, None
    return st, out[:int(off[-1])].copy(), off
