"""ctypes binding of libbfsc.so (argument marshalling only).

Every computation runs in the HIP kernels behind include/bfsc.h; this module
passes torch device pointers and sizes through, and raises when the library
is missing or a call fails.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfsc.so")

OK, E_INVAL, E_CAPACITY, E_CORRUPT, E_HIP, E_UNIMPLEMENTED = 0, 1, 2, 3, 4, 5
SEL_DEFAULT, SEL_PLAIN_BP, SEL_EXHAUSTIVE, SEL_LEARNED = -1, 0, 1, 2
RAW_BELOW = 32  # the library's default compression threshold
OP_BFS, OP_SELECT, OP_ENCODE, OP_DECODE, OP_FEATURES, OP_MLP = 0, 1, 2, 3, 4, 5
OP_ENCODE_PLACE, OP_PIPELINE = 6, 7
OP_BITMAP_ENCODE, OP_BITMAP_DECODE = 8, 9
N_PARAMS = 7011
DECODE_NOALLOC_MAX_SEGS = 65536  # BFSC_DECODE_NOALLOC_MAX_SEGS

vp = ctypes.c_void_p
u32, u64, i32, sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t


class CSR(ctypes.Structure):
    _fields_ = [("n_vertices", u32), ("n_arcs", u64), ("row_ptr", vp), ("col_idx", vp)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("ids", vp), ("seg_off", vp), ("seg_lo", vp), ("seg_hi", vp), ("seg_level", vp),
                ("nseg", u32), ("max_ids", u64)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class Tune(ctypes.Structure):
    _fields_ = [("enc_waves", u32), ("enc_wg_per_cu", u32), ("dec_waves", u32),
                ("dec_wg_per_cu", u32), ("enc_pack", u32), ("dec_mode", u32)]


class Config(ctypes.Structure):
    _fields_ = [("selector", i32), ("raw_below", u32), ("resolve_literal", u32), ("autotune", u32),
                ("tune_cache", ctypes.c_char_p)]


class PipelineBufs(ctypes.Structure):
    _fields_ = [("frontier", vp), ("frontier_len", vp), ("prev_frontier", vp),
                ("prev_frontier_len", vp), ("level", vp), ("parent", vp), ("seg_off", vp),
                ("stream", vp), ("stream_cap", sz), ("seg_byte_off", vp), ("decoded", vp),
                ("decoded_off", vp), ("classes", vp)]


P = ctypes.POINTER
_SIGS = {
    "bfsc_pipeline_create": [vp, P(CSR), vp, u32, ctypes.c_int, ctypes.c_int, P(vp)],
    "bfsc_pipeline_start": [vp, u32, vp],
    "bfsc_pipeline_step": [vp, vp, P(u32)],
    "bfsc_pipeline_buffers": [vp, P(PipelineBufs)],
    "bfsc_pipeline_destroy": [vp],
    "bfsc_memcpy": [vp, vp, sz],
    "bfsc_create": [P(vp), ctypes.c_int, P(Config)],
    "bfsc_destroy": [vp],
    "bfsc_get_config": [vp, P(Config)],
    "bfsc_workspace_size": [vp, ctypes.c_int, u64, u32, P(sz)],
    "bfsc_bfs_workspace_size": [P(CSR), P(sz)],
    "bfsc_bfs_init": [vp, P(CSR), u32, vp, vp, vp, vp, vp, vp],
    "bfsc_bfs_level": [vp, P(CSR), i32, vp, vp, vp, vp, vp, vp, vp, vp],
    "bfsc_bfs_set_direction": [vp, ctypes.c_float, ctypes.c_float],
    "bfsc_partition": [vp, vp, vp, u32, vp, vp],
    "bfsc_exchange_workspace_size": [P(CSR), u32, P(sz)],
    "bfsc_exchange_init": [vp, P(CSR), u32, vp, vp],
    "bfsc_candidates": [vp, P(CSR), vp, vp, vp, u32, vp, u64, vp, vp, vp, vp, vp],
    "bfsc_merge_filter": [vp, P(CSR), i32, vp, vp, vp, vp, vp, vp, vp, vp],
    "bfsc_select": [vp, P(BatchDesc), ctypes.c_int, vp, vp, vp, vp],
    "bfsc_encode_bound": [u64, u32, P(sz)],
    "bfsc_encode": [vp, P(BatchDesc), vp, ctypes.c_int, vp, sz, vp, vp, vp],
    "bfsc_decode": [vp, vp, vp, u32, u64, vp, u64, vp, vp, vp],
    "bfsc_decode_noalloc": [vp, vp, vp, u32, u64, vp, u64, vp, vp],
    "bfsc_bitmap_encode_bound": [u64, u32, P(sz)],
    "bfsc_bitmap_encode": [vp, vp, vp, u32, u64, vp, sz, vp, vp, vp],
    "bfsc_bitmap_decode": [vp, vp, vp, u32, u64, vp, u64, vp, vp, vp],
    "bfsc_features": [vp, P(BatchDesc), vp, vp, vp],
    "bfsc_mlp_param_count": [],
    "bfsc_mlp_init": [vp, u64],
    "bfsc_mlp_set_weights": [vp, vp],
    "bfsc_mlp_get_weights": [vp, vp],
    "bfsc_mlp_forward": [vp, vp, u32, vp, vp, vp],
    "bfsc_mlp_infer": [vp, vp, u32, vp, vp, vp],
    "bfsc_mlp_grad": [vp, vp, vp, u32, vp, vp, vp, vp],
    "bfsc_mlp_train_step": [vp, vp, vp, u32, P(Adam), vp, vp, vp],
    "bfsc_get_tune": [vp, P(Tune)],
    "bfsc_set_tune": [vp, P(Tune)],
    "bfsc_autotune": [vp, P(BatchDesc), vp, vp],
    "bfsc_sync_status": [vp, vp],
    "bfsc_timing_enable": [vp, ctypes.c_int],
    "bfsc_timing_read": [vp, ctypes.c_int, P(ctypes.c_double), P(u64)],
}

_lock = threading.Lock()
_lib = None


def load() -> ctypes.CDLL:
    """Loads libbfsc.so; raises if it has not been built.

    torch is imported first: it brings its own HIP runtime (SONAME
    libamdhip64.so.7), and the library's dependency on that SONAME must bind
    to the runtime already in the process, never to a second copy."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libbfsc.so not found at %s: build it with "
                                  "`python -m paper_1704_00513_amd.build`" % LIB_PATH)
            import torch  # noqa: F401  (loads the process's HIP runtime)
            lib = ctypes.CDLL(LIB_PATH)
            for name, args in _SIGS.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            lib.bfsc_status_string.argtypes = [ctypes.c_int]
            lib.bfsc_status_string.restype = ctypes.c_char_p
            lib.bfsc_config_default.argtypes = [P(Config)]
            lib.bfsc_config_default.restype = None
            _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS) + ["bfsc_status_string", "bfsc_config_default"]


def default_config() -> Config:
    c = Config()
    load().bfsc_config_default(ctypes.byref(c))
    return c


class BfscError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().bfsc_status_string(status).decode()
        super().__init__("%s: %s (status %d)" % (where, msg, status))


def check(status: int, where: str) -> None:
    if status != OK:
        raise BfscError(status, where)


def ptr(t) -> int | None:
    """Device (or host numpy) pointer of a tensor / array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()
