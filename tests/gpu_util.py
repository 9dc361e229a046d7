"""Helpers for the GPU parity tests: run the HIP path through the C-ABI on
host (numpy) inputs and bring results back.  Imports the product package
only; the tests compare its outputs with the oracle."""
import numpy as np


def torch():
    import torch as t
    return t


def to_dev(a, dtype_np, dtype_view):
    t = torch()
    a = np.ascontiguousarray(a, dtype_np)
    if a.size == 0:
        a = np.zeros(1, dtype_np)
    return t.from_numpy(a.view(dtype_view)).cuda()


def device_batch(b):
    """oracle.Batch -> paper_1704_00513_amd.DeviceBatch (same arrays)."""
    from paper_1704_00513_amd import DeviceBatch
    return DeviceBatch.from_host(b.ids, b.seg_off, b.seg_lo, b.seg_hi, b.seg_level)


def gpu_encode(ctx, b, classes=None, mode=1, out_cap=None):
    import paper_1704_00513_amd as P
    t = torch()
    db = device_batch(b)
    cap = P.Context.encode_bound(b.n_ids, b.nseg) if out_cap is None else out_cap
    out = t.zeros(max(4, cap), dtype=t.uint8, device="cuda")
    sbo = t.zeros(b.nseg + 1, dtype=t.int64, device="cuda")
    cls = None if classes is None else to_dev(classes, np.uint8, np.uint8)
    ctx.encode(db, out, sbo, classes=cls, mode=mode, out_cap=cap)
    st = ctx.sync_status()
    sbo_h = sbo.cpu().numpy().view(np.uint64)
    total = int(sbo_h[-1]) if st == 0 else 0
    return st, out[:total].cpu().numpy(), sbo_h


def gpu_decode(ctx, stream, sbo, max_ids=None, out_cap=None):
    t = torch()
    sbo = np.ascontiguousarray(sbo, np.uint64)
    nseg = sbo.size - 1
    data = to_dev(np.concatenate([stream, np.zeros(4, np.uint8)]), np.uint8, np.uint8)
    if max_ids is None:
        max_ids = 16 * int(sbo[-1]) + 1
    cap = max_ids if out_cap is None else out_cap
    out = t.zeros(max(1, cap), dtype=t.int32, device="cuda")
    off = t.zeros(nseg + 1, dtype=t.int64, device="cuda")
    ctx.decode(data, to_dev(sbo, np.uint64, np.int64), nseg, max_ids, out, off, out_cap=cap)
    st = ctx.sync_status()
    off_h = off.cpu().numpy().view(np.uint64)
    n = int(off_h[-1]) if st == 0 else 0
    return st, out[:n].cpu().numpy().view(np.uint32), off_h


def gpu_select(ctx, b, mode):
    t = torch()
    db = device_batch(b)
    cls = t.zeros(db.n_blocks_max, dtype=t.uint8, device="cuda")
    fb = t.zeros(1, dtype=t.int64, device="cuda")
    ctx.select(db, mode, cls, fallbacks=fb)
    st = ctx.sync_status()
    return st, cls[:b.n_blocks].cpu().numpy(), int(fb.item())


def gpu_features(ctx, b):
    t = torch()
    db = device_batch(b)
    feat = t.zeros((db.n_blocks_max, 8), dtype=t.int16, device="cuda")
    ctx.features(db, feat)
    st = ctx.sync_status()
    return st, feat[:b.n_blocks].cpu().numpy().view(np.uint16)


def shifted_batch(b, shift):
    """The batch with its IDs in a device buffer that starts `shift`
    elements into an allocation: 4-byte aligned, not 16-byte aligned.
    Returns the DeviceBatch and the allocation (keep it alive)."""
    from paper_1704_00513_amd import DeviceBatch
    t = torch()
    dev = device_batch(b)
    ids = np.ascontiguousarray(b.ids, np.uint32)
    buf = t.zeros(ids.size + shift + 4, dtype=t.int32, device="cuda")
    if ids.size:
        buf[shift:shift + ids.size] = t.from_numpy(ids.view(np.int32)).to("cuda")
    view = buf[shift:shift + max(ids.size, 1)]
    return DeviceBatch(view, dev.seg_off, dev.seg_lo, dev.seg_hi, dev.seg_level, max_ids=dev.max_ids), buf


def stream_classes(stream, sbo, seg_off):
    """The class of every block of a batch as its compressed stream records
    it (directory entries); blocks of raw and empty segments get 0, which an
    encoder skips."""
    stream = np.ascontiguousarray(stream, np.uint8)
    sizes = np.diff(np.asarray(seg_off, np.int64))
    out = []
    for r, n in enumerate(sizes):
        nb = (int(n) + 127) // 128
        s0, s1 = int(sbo[r]), int(sbo[r + 1])
        w = stream[s0:s1].view(np.uint32) if s1 > s0 else np.zeros(0, np.uint32)
        if w.size >= 4 and w[1] > w[2]:
            out.extend(int(w[4 + 2 * k + 1]) & 0xFF for k in range(nb))
        else:
            out.extend([0] * nb)
    return np.array(out, np.uint8)
