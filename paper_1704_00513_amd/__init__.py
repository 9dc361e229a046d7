"""bfsc: lossless compression of BFS frontiers on one MI355X (gfx950).

Python face of libbfsc.so (include/bfsc.h).  torch supplies device memory and
streams; every step of the path -- BFS level, partition, codec choice,
encode, decode, selector features and the MLP -- runs in this project's HIP
kernels.  Method: Romera, "Optimizing Communication by Compression for
Multi-GPU Scalable Breadth-First Searches" (arXiv 1704.00513), BFS with
compression around the frontier exchanges.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (DECODE_NOALLOC_MAX_SEGS, E_CAPACITY, E_CORRUPT, E_HIP, E_INVAL, N_PARAMS, OK, OP_DECODE, OP_ENCODE,
                   OP_FEATURES, OP_MLP, OP_SELECT, RAW_BELOW, SEL_DEFAULT, SEL_EXHAUSTIVE, SEL_LEARNED,
                   SEL_PLAIN_BP, BfscError, check, ptr)

__all__ = ["Context", "DeviceGraph", "DeviceBatch", "SEL_DEFAULT", "SEL_PLAIN_BP", "SEL_EXHAUSTIVE",
           "SEL_LEARNED", "RAW_BELOW", "DECODE_NOALLOC_MAX_SEGS", "BfscError", "OK", "E_INVAL", "E_CAPACITY", "E_CORRUPT", "E_HIP"]


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class DeviceGraph:
    """A CSR graph resident in HBM (row_ptr u64[V+1], col_idx u32[arcs])."""

    def __init__(self, row_ptr, col_idx, device="cuda"):
        torch = _torch()
        self.row_ptr = torch.from_numpy(np.ascontiguousarray(row_ptr).view(np.int64)).to(device)
        col = np.ascontiguousarray(col_idx)
        if col.size == 0:
            col = np.zeros(1, np.uint32)
        self.col_idx = torch.from_numpy(col.view(np.int32)).to(device)
        self.n_vertices = int(len(row_ptr) - 1)
        self.n_arcs = int(col_idx.size)
        self.desc = _lib.CSR(self.n_vertices, self.n_arcs, ptr(self.row_ptr), ptr(self.col_idx))

    @classmethod
    def from_host(cls, g, device="cuda"):
        return cls(g.row_ptr, g.col_idx, device)


class DeviceBatch:
    """Segments to compress: ids u32 (concatenated), seg_off u64[R+1],
    seg_lo / seg_hi u32[R], seg_level i32[R] (torch device tensors)."""

    def __init__(self, ids, seg_off, seg_lo, seg_hi, seg_level=None, max_ids=None):
        self.ids, self.seg_off, self.seg_lo, self.seg_hi = ids, seg_off, seg_lo, seg_hi
        self.seg_level = seg_level
        self.nseg = int(seg_lo.numel())
        self.max_ids = int(ids.numel() if max_ids is None else max_ids)
        self.desc = _lib.BatchDesc(ptr(ids), ptr(seg_off), ptr(seg_lo), ptr(seg_hi), ptr(seg_level),
                                   self.nseg, self.max_ids)

    @classmethod
    def from_host(cls, ids, seg_off, seg_lo, seg_hi, seg_level=None, device="cuda"):
        torch = _torch()
        t = lambda a, dt, vdt: torch.from_numpy(np.ascontiguousarray(a, dt).view(vdt)).to(device)
        ids_np = np.ascontiguousarray(ids, np.uint32)
        if ids_np.size == 0:
            ids_np = np.zeros(1, np.uint32)
        ids_t = torch.from_numpy(ids_np.view(np.int32)).to(device)
        lev = None if seg_level is None else t(seg_level, np.int32, np.int32)
        return cls(ids_t, t(seg_off, np.uint64, np.int64), t(seg_lo, np.uint32, np.int32),
                   t(seg_hi, np.uint32, np.int32), lev, max_ids=int(np.asarray(seg_off)[-1]))

    @property
    def n_blocks_max(self) -> int:
        return (self.max_ids + 127) // 128 + self.nseg


def memcpy_to_host(dev_ptr: int, count: int, dtype) -> np.ndarray:
    """Copies count elements of dtype from a device pointer (synchronous)."""
    out = np.empty(count, dtype)
    if count:
        check(_lib.load().bfsc_memcpy(out.ctypes.data, dev_ptr, out.nbytes), "bfsc_memcpy")
    return out


class Pipeline:
    """The per-level BFS + compression pipeline of one traversal (see
    bfsc_pipeline_* in bfsc.h).  use_graph replays captured HIP graphs."""

    def __init__(self, ctx: "Context", g: DeviceGraph, bounds, mode=SEL_EXHAUSTIVE,
                 use_graph: bool = True):
        self.ctx, self.g = ctx, g
        self.bounds = np.ascontiguousarray(bounds, np.uint32)
        self.nseg = self.bounds.size - 1
        h = ctypes.c_void_p()
        check(_lib.load().bfsc_pipeline_create(ctx.h, ctypes.byref(g.desc), self.bounds.ctypes.data,
                                               self.nseg, int(mode), int(use_graph), ctypes.byref(h)),
              "bfsc_pipeline_create")
        self.h = h

    def start(self, root: int, stream=None):
        check(_lib.load().bfsc_pipeline_start(self.h, int(root), _stream(stream)), "bfsc_pipeline_start")

    def step(self, stream=None, wait: bool = True):
        """One level; returns the next frontier's length when wait is set."""
        n = ctypes.c_uint32()
        check(_lib.load().bfsc_pipeline_step(self.h, _stream(stream),
                                             ctypes.byref(n) if wait else None), "bfsc_pipeline_step")
        return int(n.value) if wait else None

    def buffers(self) -> "_lib.PipelineBufs":
        b = _lib.PipelineBufs()
        check(_lib.load().bfsc_pipeline_buffers(self.h, ctypes.byref(b)), "bfsc_pipeline_buffers")
        return b

    def last_step(self):
        """Host copies of what the last step compressed and decompressed."""
        b = self.buffers()
        n = int(memcpy_to_host(b.prev_frontier_len, 1, np.uint32)[0])
        sbo = memcpy_to_host(b.seg_byte_off, self.nseg + 1, np.uint64)
        return dict(frontier=memcpy_to_host(b.prev_frontier, n, np.uint32),
                    seg_off=memcpy_to_host(b.seg_off, self.nseg + 1, np.uint64),
                    stream=memcpy_to_host(b.stream, int(sbo[-1]), np.uint8),
                    seg_byte_off=sbo,
                    decoded=memcpy_to_host(b.decoded, n, np.uint32),
                    decoded_off=memcpy_to_host(b.decoded_off, self.nseg + 1, np.uint64))

    def levels(self):
        b = self.buffers()
        return (memcpy_to_host(b.level, self.g.n_vertices, np.int32),
                memcpy_to_host(b.parent, self.g.n_vertices, np.int32))

    def close(self):
        if getattr(self, "h", None):
            _lib.load().bfsc_pipeline_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One bfsc context on one GPU, with grow-only workspaces."""

    def __init__(self, device: int = 0, selector: int | None = None, raw_below: int | None = None,
                 resolve_literal: bool | None = None, autotune: bool | None = None,
                 tune_cache: str | None = None):
        """Settings left at None keep the library's defaults (bfsc_config_default)."""
        lib = _lib.load()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("bfsc needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = device
        torch.cuda.set_device(device)
        cfg = _lib.default_config()
        if selector is not None:
            cfg.selector = int(selector)
        if raw_below is not None:
            cfg.raw_below = int(raw_below)
        if resolve_literal is not None:
            cfg.resolve_literal = int(bool(resolve_literal))
        if autotune is not None:
            cfg.autotune = int(bool(autotune))
        self._tune_cache = None if tune_cache is None else str(tune_cache).encode()
        cfg.tune_cache = self._tune_cache
        h = ctypes.c_void_p()
        check(lib.bfsc_create(ctypes.byref(h), device, ctypes.byref(cfg)), "bfsc_create")
        self.h = h
        self._ws = {}

    def config(self) -> dict:
        c = _lib.Config()
        check(_lib.load().bfsc_get_config(self.h, ctypes.byref(c)), "bfsc_get_config")
        return dict(selector=c.selector, raw_below=c.raw_below, resolve_literal=bool(c.resolve_literal),
                    autotune=bool(c.autotune), tune_cache=None if c.tune_cache is None else c.tune_cache.decode())

    def close(self):
        if getattr(self, "h", None):
            _lib.load().bfsc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- workspaces

    def _grow(self, key, nbytes):
        torch = _torch()
        t = self._ws.get(key)
        if t is None or t.numel() < nbytes:
            t = torch.empty(max(256, int(nbytes)), dtype=torch.uint8, device="cuda")
            self._ws[key] = t
        return t

    def workspace(self, op: int, max_ids: int, nseg: int, key=None):
        n = ctypes.c_size_t()
        check(_lib.load().bfsc_workspace_size(self.h, op, max_ids, nseg, ctypes.byref(n)),
              "bfsc_workspace_size")
        return self._grow(key or ("op", op), n.value)

    def bfs_workspace(self, g: DeviceGraph, key="bfs"):
        n = ctypes.c_size_t()
        check(_lib.load().bfsc_bfs_workspace_size(ctypes.byref(g.desc), ctypes.byref(n)),
              "bfsc_bfs_workspace_size")
        return self._grow(key, n.value)

    # ---------------------------------------------------------- BFS

    def bfs_init(self, g, root, level, parent, frontier, frontier_len, ws, stream=None):
        check(_lib.load().bfsc_bfs_init(self.h, ctypes.byref(g.desc), int(root), ptr(level),
                                        ptr(parent), ptr(frontier), ptr(frontier_len), ptr(ws),
                                        _stream(stream)), "bfsc_bfs_init")

    def bfs_level(self, g, cur_level, frontier, frontier_len, level, parent, nxt, next_len, ws,
                  stream=None):
        check(_lib.load().bfsc_bfs_level(self.h, ctypes.byref(g.desc), int(cur_level),
                                         ptr(frontier), ptr(frontier_len), ptr(level), ptr(parent),
                                         ptr(nxt), ptr(next_len), ptr(ws), _stream(stream)),
              "bfsc_bfs_level")

    def bfs_set_direction(self, alpha: float = 14.0, beta: float = 24.0):
        """Direction-optimizing BFS levels (alpha = 0: top-down only)."""
        check(_lib.load().bfsc_bfs_set_direction(self.h, float(alpha), float(beta)), "bfsc_bfs_set_direction")

    def partition(self, ids, n_dev, bounds, seg_off, stream=None):
        check(_lib.load().bfsc_partition(ptr(ids), ptr(n_dev), ptr(bounds), int(bounds.numel()) - 1,
                                         ptr(seg_off), _stream(stream)), "bfsc_partition")

    # ---------------------------------------------------------- candidate exchange

    def exchange_workspace(self, g: DeviceGraph, nseg: int, key="exchange"):
        n = ctypes.c_size_t()
        check(_lib.load().bfsc_exchange_workspace_size(ctypes.byref(g.desc), int(nseg), ctypes.byref(n)),
              "bfsc_exchange_workspace_size")
        return self._grow(key, n.value)

    def exchange_init(self, g, nseg, ws, stream=None):
        check(_lib.load().bfsc_exchange_init(self.h, ctypes.byref(g.desc), int(nseg), ptr(ws), _stream(stream)),
              "bfsc_exchange_init")

    def candidates(self, g, frontier, frontier_len, bounds, ids, seg_off, seg_lo, seg_hi, ws, cap=None,
                   stream=None):
        nseg = int(bounds.numel()) - 1
        cap = ids.numel() if cap is None else cap
        check(_lib.load().bfsc_candidates(self.h, ctypes.byref(g.desc), ptr(frontier), ptr(frontier_len),
                                          ptr(bounds), nseg, ptr(ids), int(cap), ptr(seg_off), ptr(seg_lo),
                                          ptr(seg_hi), ptr(ws), _stream(stream)), "bfsc_candidates")

    def merge_filter(self, g, cur_level, ids, n_dev, level, nxt, next_len, bfs_ws, ws, stream=None):
        check(_lib.load().bfsc_merge_filter(self.h, ctypes.byref(g.desc), int(cur_level), ptr(ids), ptr(n_dev),
                                            ptr(level), ptr(nxt), ptr(next_len), ptr(bfs_ws), ptr(ws),
                                            _stream(stream)), "bfsc_merge_filter")

    # ---------------------------------------------------------- codec

    def select(self, b: DeviceBatch, mode, classes, fallbacks=None, ws=None, stream=None):
        ws = ws if ws is not None else self.workspace(OP_SELECT, b.max_ids, b.nseg)
        check(_lib.load().bfsc_select(self.h, ctypes.byref(b.desc), int(mode), ptr(classes),
                                      ptr(fallbacks), ptr(ws), _stream(stream)), "bfsc_select")

    def features(self, b: DeviceBatch, feat, ws=None, stream=None):
        ws = ws if ws is not None else self.workspace(OP_FEATURES, b.max_ids, b.nseg)
        check(_lib.load().bfsc_features(self.h, ctypes.byref(b.desc), ptr(feat), ptr(ws),
                                        _stream(stream)), "bfsc_features")

    @staticmethod
    def encode_bound(n_ids: int, nseg: int) -> int:
        n = ctypes.c_size_t()
        check(_lib.load().bfsc_encode_bound(n_ids, nseg, ctypes.byref(n)), "bfsc_encode_bound")
        return n.value

    def encode(self, b: DeviceBatch, out, seg_byte_off, classes=None, mode=SEL_EXHAUSTIVE,
               ws=None, stream=None, out_cap=None):
        ws = ws if ws is not None else self.workspace(OP_ENCODE, b.max_ids, b.nseg)
        cap = out.numel() * out.element_size() if out_cap is None else out_cap
        check(_lib.load().bfsc_encode(self.h, ctypes.byref(b.desc), ptr(classes), int(mode), ptr(out),
                                      cap, ptr(seg_byte_off), ptr(ws), _stream(stream)), "bfsc_encode")

    def decode(self, data, seg_byte_off, nseg, max_ids, out_ids, out_off, ws=None, stream=None,
               out_cap=None):
        ws = ws if ws is not None else self.workspace(OP_DECODE, max_ids, nseg)
        cap = out_ids.numel() if out_cap is None else out_cap
        check(_lib.load().bfsc_decode(self.h, ptr(data), ptr(seg_byte_off), int(nseg), int(max_ids),
                                      ptr(out_ids), cap, ptr(out_off), ptr(ws), _stream(stream)),
              "bfsc_decode")

    def decode_noalloc(self, data, seg_byte_off, nseg, max_ids, out_ids, out_off, stream=None,
                       out_cap=None):
        """bfsc_decode with the library's fixed scratch array instead of a
        workspace (at most DECODE_NOALLOC_MAX_SEGS segments)."""
        cap = out_ids.numel() if out_cap is None else out_cap
        check(_lib.load().bfsc_decode_noalloc(self.h, ptr(data), ptr(seg_byte_off), int(nseg), int(max_ids),
                                              ptr(out_ids), cap, ptr(out_off), _stream(stream)),
              "bfsc_decode_noalloc")

    # ---------------------------------------------------------- bitmap codec

    @staticmethod
    def bitmap_encode_bound(n_words: int, nseg: int) -> int:
        n = ctypes.c_size_t()
        check(_lib.load().bfsc_bitmap_encode_bound(n_words, nseg, ctypes.byref(n)), "bfsc_bitmap_encode_bound")
        return n.value

    def bitmap_encode(self, bits, seg_w, nseg, max_words, out, seg_byte_off, ws=None, stream=None, out_cap=None):
        """Bitmap codec: words bits (u32 tensor), segments seg_w (u64 word
        ranges, nseg + 1) -> out bytes, seg_byte_off (nseg + 1)."""
        ws = ws if ws is not None else self.workspace(_lib.OP_BITMAP_ENCODE, max_words, nseg)
        cap = out.numel() * out.element_size() if out_cap is None else out_cap
        check(_lib.load().bfsc_bitmap_encode(self.h, ptr(bits), ptr(seg_w), int(nseg), int(max_words), ptr(out),
                                             cap, ptr(seg_byte_off), ptr(ws), _stream(stream)),
              "bfsc_bitmap_encode")

    def bitmap_decode(self, data, seg_byte_off, nseg, max_words, out, out_off, ws=None, stream=None,
                      out_cap=None):
        ws = ws if ws is not None else self.workspace(_lib.OP_BITMAP_DECODE, max_words, nseg)
        cap = out.numel() if out_cap is None else out_cap
        check(_lib.load().bfsc_bitmap_decode(self.h, ptr(data), ptr(seg_byte_off), int(nseg), int(max_words),
                                             ptr(out), cap, ptr(out_off), ptr(ws), _stream(stream)),
              "bfsc_bitmap_decode")

    def sync_status(self, stream=None) -> int:
        return _lib.load().bfsc_sync_status(self.h, _stream(stream))

    def sync(self, stream=None) -> None:
        check(self.sync_status(stream), "kernel status")

    # ---------------------------------------------------------- timing

    def timing(self, enable: bool = True) -> None:
        check(_lib.load().bfsc_timing_enable(self.h, int(enable)), "bfsc_timing_enable")

    def timing_read(self, op: int):
        """-> (total milliseconds, launches) of op's main kernel since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_uint64()
        check(_lib.load().bfsc_timing_read(self.h, op, ctypes.byref(ms), ctypes.byref(n)),
              "bfsc_timing_read")
        return ms.value, n.value

    # ---------------------------------------------------------- tuning

    def get_tune(self):
        t = _lib.Tune()
        check(_lib.load().bfsc_get_tune(self.h, ctypes.byref(t)), "bfsc_get_tune")
        return dict(enc_waves=t.enc_waves, enc_wg_per_cu=t.enc_wg_per_cu, dec_waves=t.dec_waves,
                    dec_wg_per_cu=t.dec_wg_per_cu, enc_pack=t.enc_pack, dec_mode=t.dec_mode)

    def set_tune(self, **kw):
        cur = self.get_tune()
        cur.update(kw)
        t = _lib.Tune(cur["enc_waves"], cur["enc_wg_per_cu"], cur["dec_waves"], cur["dec_wg_per_cu"],
                      cur["enc_pack"], cur["dec_mode"])
        check(_lib.load().bfsc_set_tune(self.h, ctypes.byref(t)), "bfsc_set_tune")

    def autotune(self, b: "DeviceBatch", ws=None, stream=None):
        """Measures the launch shapes on a sample batch and keeps the fastest."""
        ws = ws if ws is not None else self.workspace(OP_ENCODE, b.max_ids, b.nseg)
        check(_lib.load().bfsc_autotune(self.h, ctypes.byref(b.desc), ptr(ws), _stream(stream)),
              "bfsc_autotune")
        return self.get_tune()

    # ---------------------------------------------------------- MLP

    def mlp_init(self, seed: int):
        """He-uniform initial parameters from the counter RNG (bfsc_mlp_init)."""
        check(_lib.load().bfsc_mlp_init(self.h, int(seed)), "bfsc_mlp_init")

    def mlp_set_weights(self, params: np.ndarray):
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == N_PARAMS
        check(_lib.load().bfsc_mlp_set_weights(self.h, p.ctypes.data), "bfsc_mlp_set_weights")

    def mlp_get_weights(self) -> np.ndarray:
        p = np.empty(N_PARAMS, np.float32)
        check(_lib.load().bfsc_mlp_get_weights(self.h, p.ctypes.data), "bfsc_mlp_get_weights")
        return p

    def mlp_forward(self, X, n, logits, stream=None):
        check(_lib.load().bfsc_mlp_forward(self.h, ptr(X), int(n), ptr(logits), None, _stream(stream)),
              "bfsc_mlp_forward")

    def mlp_grad(self, X, y, n, grads, loss=None, ws=None, stream=None):
        ws = ws if ws is not None else self.workspace(OP_MLP, n, 0, key="mlp")
        check(_lib.load().bfsc_mlp_grad(self.h, ptr(X), ptr(y), int(n), ptr(grads), ptr(loss), ptr(ws),
                                        _stream(stream)), "bfsc_mlp_grad")

    def mlp_infer(self, X, n, logits=None, classes=None, stream=None):
        """Logits and/or predicted classes from the matrix-core inference kernel."""
        check(_lib.load().bfsc_mlp_infer(self.h, ptr(X), int(n), ptr(logits), ptr(classes),
                                         _stream(stream)), "bfsc_mlp_infer")

    def mlp_train_step(self, X, y, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss=None, ws=None,
                       stream=None):
        ws = ws if ws is not None else self.workspace(OP_MLP, n, 0, key="mlp")
        opt = _lib.Adam(lr, beta1, beta2, eps)
        check(_lib.load().bfsc_mlp_train_step(self.h, ptr(X), ptr(y), int(n), ctypes.byref(opt),
                                              ptr(loss), ptr(ws), _stream(stream)),
              "bfsc_mlp_train_step")
