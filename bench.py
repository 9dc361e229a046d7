"""Frontier-codec benchmark on one MI355X.

Workload (default): the full pipeline at the largest one-GPU size.  R-MAT
scale 26 (67.1 M vertices), edge factor 16, (a, b, c, d) = (0.57, 0.19, 0.19,
0.05), seed 1; direction-optimizing BFS on the GPU from 16 seeded roots; every
level's frontier split by vertex-ID range into 1024 segments whose sizes are
Zipf(1.2) draws over 1..2^20 normalised to the vertex range; the batch of all
segments of all levels of all roots is resident in HBM.  One step = one encode
of the whole batch with the learned codec choice (the trained network on the
matrix cores inside the pack pass, exhaustive fallback where its pick is
invalid) followed by its decode.  The exhaustive choice is timed beside it.

value = raw frontier bytes (4 B per ID) / (encode + decode time), GB/s.
The JSON line also carries the roofline of the dominant kernel (algorithmic
bytes per launch / its HIP-event-timed duration, against 8 TB/s), the
whole-step fraction of HBM peak on algorithmic bytes, and the CPU oracle
timed on a bounded sample on this host.

    python bench.py [--steps 10] [--warmup 3] [--scale 26] [--roots 16] [--nseg 1024]
                    [--bounds zipf] [--mode learned]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("codec.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1704_00513_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_source_sha()
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        kv = dict(x.split("=", 1) for x in line.split())
        if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("sha") == sha:
            return float(kv["bytes_per_launch"])
    return None


def build_batch(ctx, P, torch, g, roots, nseg, bounds_kind, seed):
    """GPU BFS from each root; every level's frontier goes into one device
    buffer and is partitioned on the GPU into nseg vertex ranges."""
    import inputs
    V = g.n_vertices
    dg = P.DeviceGraph.from_host(g)
    cap = V * (len(roots) + 1)
    all_ids = torch.empty(cap, dtype=torch.int32, device="cuda")
    level = torch.empty(V, dtype=torch.int32, device="cuda")
    parent = torch.empty(V, dtype=torch.int32, device="cuda")
    la = torch.zeros(1, dtype=torch.int32, device="cuda")
    lb = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = ctx.bfs_workspace(dg)
    if bounds_kind == "zipf":
        bounds_h, _ = inputs.bounds_zipf(V, nseg, seed)
    else:
        bounds_h = inputs.bounds_equal(V, nseg)
    bounds = torch.from_numpy(bounds_h.view(np.int32)).cuda()
    seg_off_l = torch.zeros(nseg + 1, dtype=torch.int64, device="cuda")
    offs, los, his, levs = [np.zeros(1, np.uint64)], [], [], []
    base = 0
    bfs_ms, bfs_levels, edges = 0.0, 0, 0
    ctx.timing(True)
    for root in roots:
        front = all_ids[base:]
        ctx.bfs_init(dg, int(root), level, parent, front, la, ws)
        L = 0
        while True:
            n = int(la.item())
            if n == 0:
                break
            ctx.partition(front, la, bounds, seg_off_l)
            so = seg_off_l.cpu().numpy().view(np.uint64) + np.uint64(base)
            offs.append(so[1:])
            los.append(bounds_h[:-1])
            his.append(bounds_h[1:])
            levs.append(np.full(nseg, L, np.int32))
            nxt = all_ids[base + n:]
            ctx.bfs_level(dg, L, front, la, level, parent, nxt, lb, ws)
            base += n
            front = nxt
            la, lb = lb, la
            L += 1
        bfs_levels += L
        lv = level.cpu().numpy()
        deg = np.diff(g.row_ptr)
        edges += int(deg[lv >= 0].sum())
        ms, cnt = ctx.timing_read(P._lib.OP_BFS)
        bfs_ms += ms
    ctx.timing(False)
    ctx.sync()
    seg_off = np.concatenate(offs)
    b = P.DeviceBatch(all_ids[:max(1, base)],
                      torch.from_numpy(seg_off.view(np.int64)).cuda(),
                      torch.from_numpy(np.concatenate(los).view(np.int32)).cuda(),
                      torch.from_numpy(np.concatenate(his).view(np.int32)).cuda(),
                      torch.from_numpy(np.concatenate(levs)).cuda(), max_ids=base)
    host = dict(seg_off=seg_off, seg_lo=np.concatenate(los), seg_hi=np.concatenate(his),
                seg_level=np.concatenate(levs))
    return b, host, dict(bfs_ms=bfs_ms, bfs_levels=bfs_levels, edges=edges, n_ids=base)


def save_batch(b, host, bfs, path):
    """The frontier batch (host copies) and its BFS figures, as .npy files."""
    os.makedirs(path, exist_ok=True)
    np.save(os.path.join(path, "ids.npy"), b.ids[:max(1, b.max_ids)].cpu().numpy().view(np.uint32))
    for k in ("seg_off", "seg_lo", "seg_hi", "seg_level"):
        np.save(os.path.join(path, k + ".npy"), host[k])
    with open(os.path.join(path, "meta.json"), "w") as f:
        json.dump(bfs, f)


def load_batch(P, torch, path):
    ld = lambda k: np.load(os.path.join(path, k + ".npy"), allow_pickle=False)
    host = {k: ld(k) for k in ("seg_off", "seg_lo", "seg_hi", "seg_level")}
    bfs = json.load(open(os.path.join(path, "meta.json")))
    ids = np.load(os.path.join(path, "ids.npy"), mmap_mode="r", allow_pickle=False)
    ids_t = torch.from_numpy(np.ascontiguousarray(ids).view(np.int32)).cuda()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    b = P.DeviceBatch(ids_t, t(host["seg_off"].view(np.int64)), t(host["seg_lo"].view(np.int32)),
                      t(host["seg_hi"].view(np.int32)), t(host["seg_level"].astype(np.int32)),
                      max_ids=bfs["n_ids"])
    return b, host, bfs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--graph", choices=["rmat", "uniform"], default="rmat")
    ap.add_argument("--roots", type=int, default=16)
    ap.add_argument("--nseg", type=int, default=1024)
    ap.add_argument("--bounds", choices=["equal", "zipf"], default="zipf")
    ap.add_argument("--mode", choices=["exhaustive", "plain", "learned"], default="learned",
                    help="codec choice: exhaustive search, plain minimal width, or the trained "
                         "selector (exhaustive fallback where its choice is invalid)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--bfs", choices=["do", "td"], default="do",
                    help="BFS producing the frontiers: direction-optimizing (alpha 14, beta 24) or top-down only")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--calib", action="store_true",
                    help="also run a copy-like kernel of known size (counter calibration)")
    ap.add_argument("--tune", action="append", default=[],
                    help="launch shape override, e.g. --tune enc_waves=8 --tune enc_pack=1")
    ap.add_argument("--autotune", action="store_true", help="measure launch shapes on the batch first")
    ap.add_argument("--batch-cache", default=None,
                    help="directory keeping the frontier batch between runs (written on the first run, "
                         "loaded by later ones: profiler passes skip graph generation and BFS)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import inputs
    import paper_1704_00513_amd as P

    mode = {"exhaustive": P.SEL_EXHAUSTIVE, "plain": P.SEL_PLAIN_BP, "learned": P.SEL_LEARNED}[args.mode]
    kind = inputs.RMAT if args.graph == "rmat" else inputs.UNIFORM
    workload = "rmat-s%d" % args.scale if args.graph == "rmat" else "uniform-s%d" % args.scale
    workload += "-%droots-%s%d-%s" % (args.roots, args.bounds, args.nseg, args.mode)
    graph_state = {}

    def get_graph():
        if "g" not in graph_state:
            t0 = time.time()
            g = inputs.graph(kind, args.scale, 16, args.seed)
            log("graph %s scale %d: V=%d arcs=%d (%.1fs)" % (args.graph, args.scale, g.n_vertices,
                                                            g.n_arcs, time.time() - t0))
            graph_state["g"] = g
            graph_state["roots"] = inputs.roots(g, args.roots, args.seed)
        return graph_state["g"], graph_state["roots"]

    ctx = P.Context(0)
    if args.bfs == "do":
        ctx.bfs_set_direction(14.0, 24.0)
    # the batch does not depend on the selector: one cache entry per graph,
    # roots and segment split
    cache_dir = None
    if args.batch_cache:
        cache_dir = os.path.join(args.batch_cache, workload.rsplit("-", 1)[0] + "-" + args.bfs)
    if cache_dir and os.path.exists(os.path.join(cache_dir, "meta.json")):
        b, host, bfs = load_batch(P, torch, cache_dir)
        log("batch loaded from %s" % cache_dir)
    else:
        g, roots = get_graph()
        b, host, bfs = build_batch(ctx, P, torch, g, roots, args.nseg, args.bounds, args.seed)
        if cache_dir:
            save_batch(b, host, bfs, cache_dir)
    N = bfs["n_ids"]
    log("batch: %d IDs in %d segments, %d levels; BFS %.2f ms total" % (N, b.nseg, bfs["bfs_levels"],
                                                                       bfs["bfs_ms"]))

    cap = P.Context.encode_bound(N, b.nseg)
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    sbo = torch.zeros(b.nseg + 1, dtype=torch.int64, device="cuda")
    dec = torch.empty(max(1, N), dtype=torch.int32, device="cuda")
    doff = torch.zeros(b.nseg + 1, dtype=torch.int64, device="cuda")
    ws_e = ctx.workspace(P.OP_ENCODE, b.max_ids, b.nseg)
    ws_d = ctx.workspace(P.OP_DECODE, b.max_ids, b.nseg)

    cls = None
    if mode == P.SEL_LEARNED:
        wpath = os.path.join(ROOT, "paper_1704_00513_amd", "selector_weights.npy")
        if not os.path.exists(wpath):
            sys.exit("--mode learned needs the trained selector (python -m paper_1704_00513_amd.train)")
        ctx.mlp_set_weights(np.load(wpath, allow_pickle=False))
        cls = torch.zeros(b.n_blocks_max, dtype=torch.uint8, device="cuda")
        fb = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws_s = ctx.workspace(P.OP_SELECT, b.max_ids, b.nseg)

    def step():
        # the learned choice runs inside the pack pass (matrix-core inference
        # per unit of 8 blocks)
        ctx.encode(b, out, sbo, mode=mode, ws=ws_e)
        ctx.decode(out, sbo, b.nseg, N, dec, doff, ws=ws_d)

    if args.tune:
        ctx.set_tune(**{k: int(v) for k, v in (x.split("=", 1) for x in args.tune)})
    if args.autotune:
        log("autotune:", ctx.autotune(b))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms_step = wall * 1e3 / args.steps
    st = ctx.sync_status()
    assert st == 0, "kernel status %d" % st
    value = 4.0 * N / (ms_step * 1e-3) / 1e9

    # parity at full size, on the last timed step's output: round trip exact,
    # sampled segments byte-equal to the oracle
    assert torch.equal(dec[:N], b.ids[:N]), "round trip differs"
    sbo_h = sbo.cpu().numpy().view(np.uint64)
    comp = int(sbo_h[-1])
    if cls is not None:
        # the classes of the separate selection pass, for the oracle check
        # (the fused pass picks the same ones)
        ctx.select(b, P.SEL_LEARNED, cls, fallbacks=fb, ws=ws_s)
        ctx.sync()
    check_segments(out, sbo_h, b, host, mode, cls=None if cls is None else cls.cpu().numpy())
    levels = ratio_per_level(sbo_h, host)
    # the per-kernel timing below starts warm again
    for _ in range(args.warmup):
        step()

    # per-kernel durations from event pairs around the main kernels
    ctx.timing(True)
    for _ in range(args.steps):
        step()
    ctx.sync()
    enc_ms, enc_n = ctx.timing_read(P.OP_ENCODE)
    place_ms, place_n = ctx.timing_read(P._lib.OP_ENCODE_PLACE)
    dec_ms, dec_n = ctx.timing_read(P.OP_DECODE)
    ctx.timing(False)
    enc_avg, dec_avg = enc_ms / enc_n, dec_ms / dec_n
    place_avg = place_ms / max(1, place_n)
    # algorithmic bytes per launch: the pack pass reads the raw IDs and writes
    # the compressed content; the decoder reads it and writes the raw IDs
    alg_bytes = 4.0 * N + comp
    pack_kernel = "k_enc_pack_l" if mode == P.SEL_LEARNED else "k_enc_pack_u"
    dom = (pack_kernel, enc_avg) if enc_avg >= dec_avg else ("k_decode_u", dec_avg)
    achieved = alg_bytes / (dom[1] * 1e-3) / 1e9
    traffic = read_traffic(dom[0], workload)

    res = {
        "metric": "frontier codec GB/s (enc+dec, raw bytes)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded R-MAT / uniform graphs, GPU BFS frontiers)",
        "config": {"workload": workload, "scale": args.scale, "edgefactor": 16, "roots": args.roots,
                   "segments_per_level": args.nseg, "bounds": args.bounds, "selector": args.mode,
                   "n_ids": N, "segments": b.nseg, "levels": bfs["bfs_levels"],
                   "tune": ctx.get_tune()},
        "ratio": round(4.0 * N / comp, 4),
        "ratio_per_level": levels,
        "compressed_bytes": comp,
        "encode_ms": round(enc_avg, 4),
        "encode_place_ms": round(place_avg, 4),
        "decode_ms": round(dec_avg, 4),
        "encode_GBps_raw": round(4.0 * N / (enc_avg + place_avg) / 1e6, 1),
        "decode_GBps_raw": round(4.0 * N / dec_avg / 1e6, 1),
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "alg_bytes_per_launch": int(alg_bytes)},
        # the whole step (every kernel of encode and decode, and the gaps
        # between them): algorithmic bytes of both directions over the
        # wall-clock step time
        "enc_dec_alg_frac": round((2 * alg_bytes) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "main_kernels_ms": {"pack": round(enc_avg, 4), "place": round(place_avg, 4),
                            "decode": round(dec_avg, 4),
                            "rest_of_step": round(ms_step - enc_avg - place_avg - dec_avg, 4)},
        "bfs": {"direction": args.bfs, "ms_total": round(bfs["bfs_ms"], 3), "levels": bfs["bfs_levels"],
                "GTEPS": round(bfs["edges"] / 2 / (bfs["bfs_ms"] * 1e-3) / 1e9, 3)},
    }
    if args.calib:
        # a plain elementwise kernel of known traffic (256 MiB read + 256 MiB
        # written per launch), for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE
        x = torch.zeros(1 << 26, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.add(x, 1, out=y)
        torch.cuda.synchronize()
    if not args.no_extra:
        g, roots = get_graph()
        res["extra"] = extras(ctx, P, torch, g, roots, b, host, N, comp, ms_step, args, mode)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(b, host, args.cpu_seconds, mode)
        res["cpu_baseline_all_cores"] = cpu_baseline_threads(b, host, args.cpu_seconds, mode)
    print(json.dumps(res), flush=True)
    ctx.close()


def extras(ctx, P, torch, g, roots, b, host, N, comp, ms_step, args, mode):
    """Comparison legs on the same batch: learned selector vs exhaustive, one
    launch per segment vs one batched launch, per-level pipeline replayed
    from HIP graphs vs launched kernel by kernel."""
    out = {}
    cap = P.Context.encode_bound(N, b.nseg)
    buf = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    sbo = torch.zeros(b.nseg + 1, dtype=torch.int64, device="cuda")
    dec = torch.empty(max(1, N), dtype=torch.int32, device="cuda")
    doff = torch.zeros(b.nseg + 1, dtype=torch.int64, device="cuda")
    steps = max(3, args.steps // 2)

    # learned selector (weights trained by paper_1704_00513_amd/train.py)
    wpath = os.path.join(ROOT, "paper_1704_00513_amd", "selector_weights.npy")
    if mode == P.SEL_LEARNED:
        def xstep():
            ctx.encode(b, buf, sbo, mode=P.SEL_EXHAUSTIVE)
            ctx.decode(buf, sbo, b.nseg, N, dec, doff)

        xstep()
        ctx.sync()
        assert torch.equal(dec[:N], b.ids[:N]), "exhaustive round trip differs"
        xcomp = int(sbo[-1].item())
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            xstep()
        torch.cuda.synchronize()
        xms = (time.perf_counter() - t) * 1e3 / steps
        out["exhaustive"] = {"value_GBps": round(4.0 * N / (xms * 1e-3) / 1e9, 2),
                             "ms_per_step": round(xms, 4), "compressed_bytes": xcomp,
                             "learned_size_gap_pct": round(100.0 * (comp - xcomp) / xcomp, 3),
                             "learned_vs_exhaustive_speed": round(xms / ms_step, 3)}
        # the two-pass form: a selection pass writes the class vector, then the
        # encoder reads it
        cls2 = torch.zeros(b.n_blocks_max, dtype=torch.uint8, device="cuda")
        fb2 = torch.zeros(1, dtype=torch.int64, device="cuda")

        def tstep():
            ctx.select(b, P.SEL_LEARNED, cls2, fallbacks=fb2)
            ctx.encode(b, buf, sbo, classes=cls2)
            ctx.decode(buf, sbo, b.nseg, N, dec, doff)

        tstep()
        ctx.sync()
        assert int(sbo[-1].item()) == comp, "two-pass learned size differs from the fused one"
        fb2.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            tstep()
        torch.cuda.synchronize()
        tms = (time.perf_counter() - t) * 1e3 / steps
        nblk = int(sum((np.diff(host["seg_off"].astype(np.int64)) + 127) // 128))
        out["learned_two_pass"] = {"value_GBps": round(4.0 * N / (tms * 1e-3) / 1e9, 2),
                                   "ms_per_step": round(tms, 4),
                                   "fallback_rate": round(int(fb2.item()) / steps / max(1, nblk), 5)}
    elif os.path.exists(wpath):
        ctx.mlp_set_weights(np.load(wpath, allow_pickle=False))
        cls = torch.zeros(b.n_blocks_max, dtype=torch.uint8, device="cuda")
        fb = torch.zeros(1, dtype=torch.int64, device="cuda")

        def lstep():
            ctx.encode(b, buf, sbo, mode=P.SEL_LEARNED)
            ctx.decode(buf, sbo, b.nseg, N, dec, doff)

        lstep()
        ctx.sync()
        assert torch.equal(dec[:N], b.ids[:N]), "learned round trip differs"
        lcomp = int(sbo[-1].item())
        # fallbacks are counted by the separate selection pass
        ctx.select(b, P.SEL_LEARNED, cls, fallbacks=fb)
        ctx.sync()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            lstep()
        torch.cuda.synchronize()
        lms = (time.perf_counter() - t) * 1e3 / steps
        ctx.sync()
        nblk = int(sum((np.diff(host["seg_off"].astype(np.int64)) + 127) // 128))
        out["learned"] = {"value_GBps": round(4.0 * N / (lms * 1e-3) / 1e9, 2),
                          "ms_per_step": round(lms, 4),
                          "compressed_bytes": lcomp,
                          "size_gap_vs_exhaustive_pct": round(100.0 * (lcomp - comp) / comp, 3),
                          "fallback_rate": round(int(fb.item()) / max(1, nblk), 5),
                          "vs_exhaustive_speed": round(ms_step / lms, 3)}

    # one launch per segment (the same kernels, a one-segment batch each); on
    # batches with more than 4096 non-empty segments, a seeded sample of 4096
    # of them, and the rate compared with the batched one over the same IDs
    segs = []
    so = host["seg_off"]
    nonempty = np.nonzero(np.diff(so.astype(np.int64)))[0]
    sampled = nonempty.size > 4096
    if sampled:
        nonempty = np.sort(np.random.default_rng(3).choice(nonempty, 4096, replace=False))
    for r in nonempty:
        s, e = int(so[r]), int(so[r + 1])
        sb = P.DeviceBatch(b.ids[s:e], torch.tensor([0, e - s], dtype=torch.int64, device="cuda"),
                           b.seg_lo[r:r + 1], b.seg_hi[r:r + 1], b.seg_level[r:r + 1], max_ids=e - s)
        o = torch.zeros(P.Context.encode_bound(e - s, 1), dtype=torch.uint8, device="cuda")
        segs.append((sb, o, torch.zeros(2, dtype=torch.int64, device="cuda"), dec[s:e],
                     torch.zeros(2, dtype=torch.int64, device="cuda"), e - s))
    ws_e = ctx.workspace(P.OP_ENCODE, max(x[5] for x in segs), 1, key="perseg_e")
    ws_d = ctx.workspace(P.OP_DECODE, max(x[5] for x in segs), 1, key="perseg_d")

    # the plain single-segment form: exhaustive choice, one launch per segment
    seg_mode = P.SEL_EXHAUSTIVE if mode == P.SEL_LEARNED else mode

    def pstep():
        for sb, o, sbo1, d, doff1, n in segs:
            ctx.encode(sb, o, sbo1, mode=seg_mode, ws=ws_e)
            ctx.decode(o, sbo1, 1, n, d, doff1, ws=ws_d)

    pstep()
    ctx.sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        pstep()
    torch.cuda.synchronize()
    pms = (time.perf_counter() - t) * 1e3 / 3
    nseg_ids = sum(x[5] for x in segs)
    pg = 4.0 * nseg_ids / (pms * 1e-3) / 1e9
    out["per_segment_launches"] = {"segments": len(segs), "sampled": bool(sampled), "ids": int(nseg_ids),
                                   "ms_per_step": round(pms, 3), "value_GBps": round(pg, 2),
                                   "batched_speedup": round(4.0 * N / (ms_step * 1e-3) / 1e9 / pg, 2)}

    out["per_level_root0"] = per_level(ctx, P, torch, b, host, mode)
    if args.bfs == "do":
        out["bfs_top_down_only"] = bfs_top_down(ctx, P, torch, g, roots, host)
    out["exchange_root0"] = exchange_leg(ctx, P, torch, g, int(roots[0]), host, args.nseg, mode)
    out["mall_cold"] = mall_cold(ctx, P, torch, b, buf, sbo, dec, doff, N, mode, steps)
    out["bitmap_root0"] = bitmap_leg(ctx, P, torch, g, int(roots[0]))

    # per-level pipeline for the first root: graph replay vs eager launches
    dg = P.DeviceGraph.from_host(g)
    bounds = host["seg_hi"][:args.nseg]
    bounds = np.concatenate([[host["seg_lo"][0]], bounds]).astype(np.uint32)
    for use_graph in (True, False):
        pipe = P.Pipeline(ctx, dg, bounds, mode=mode, use_graph=use_graph)
        times = []
        for rep in range(3):
            pipe.start(int(roots[0]))
            torch.cuda.synchronize()
            t = time.perf_counter()
            L, n = 0, 1
            while n:
                n = pipe.step()
                L += 1
            times.append((time.perf_counter() - t) * 1e3)
        ctx.sync()
        pipe.close()
        key = "pipeline_graph" if use_graph else "pipeline_eager"
        out[key] = {"levels": L, "ms_traversal": round(min(times), 3),
                    "us_per_level": round(1e3 * min(times) / L, 1)}
    return out


def bfs_top_down(ctx, P, torch, g, roots, host):
    """The same traversals with top-down levels only (the frontiers, and so
    the batch, are the same; checked by level count and frontier sizes)."""
    V = g.n_vertices
    dg = P.DeviceGraph.from_host(g)
    i32 = dict(dtype=torch.int32, device="cuda")
    level, parent = torch.empty(V, **i32), torch.empty(V, **i32)
    fa, fb = torch.empty(V, **i32), torch.empty(V, **i32)
    la, lb = torch.zeros(1, **i32), torch.zeros(1, **i32)
    ws = ctx.bfs_workspace(dg, key="bfs_td")
    ctx.bfs_set_direction(0.0, 0.0)
    sizes, ms, edges = [], 0.0, 0
    deg = np.diff(g.row_ptr)
    ctx.timing(True)
    for root in roots:
        ctx.bfs_init(dg, int(root), level, parent, fa, la, ws)
        L = 0
        while True:
            n = int(la.item())
            if n == 0:
                break
            sizes.append(n)
            ctx.bfs_level(dg, L, fa, la, level, parent, fb, lb, ws)
            fa, fb, la, lb = fb, fa, lb, la
            L += 1
        edges += int(deg[level.cpu().numpy() >= 0].sum())
        ms += ctx.timing_read(P._lib.OP_BFS)[0]
    ctx.timing(False)
    ctx.bfs_set_direction(14.0, 24.0)
    so = host["seg_off"].astype(np.int64)
    nseg = host["seg_lo"].size // max(1, len(sizes))
    want = [int(so[(i + 1) * nseg] - so[i * nseg]) for i in range(len(sizes))] if nseg else []
    assert sizes == want, "top-down frontiers differ from the direction-optimizing ones"
    return {"ms_total": round(ms, 3), "levels": len(sizes), "GTEPS": round(edges / 2 / (ms * 1e-3) / 1e9, 3)}


def per_level(ctx, P, torch, b, host, mode, reps=10):
    """The first root's levels, one batch per level: IDs, ratio, enc+dec time
    and rate, and the exhaustive class histogram (bitmap / bit-pack / PFOR)."""
    lev, so = host["seg_level"], host["seg_off"].astype(np.int64)
    end0 = next((i for i in range(1, lev.size) if lev[i] < lev[i - 1]), lev.size)
    res = []
    for L in np.unique(lev[:end0]):
        idx = np.nonzero(lev[:end0] == L)[0]
        r0, r1 = int(idx[0]), int(idx[-1]) + 1
        s, e = int(so[r0]), int(so[r1])
        if e == s:
            continue
        n = e - s
        sb = P.DeviceBatch(b.ids[s:e], torch.from_numpy(so[r0:r1 + 1] - s).cuda(), b.seg_lo[r0:r1],
                           b.seg_hi[r0:r1], b.seg_level[r0:r1], max_ids=n)
        nseg = r1 - r0
        cls = torch.zeros(sb.n_blocks_max, dtype=torch.uint8, device="cuda")
        ctx.select(sb, P.SEL_EXHAUSTIVE, cls)
        nblk = int(sum((np.diff(so[r0:r1 + 1]) + 127) // 128))
        c = np.bincount(cls[:nblk].cpu().numpy(), minlength=35)
        o = torch.zeros(P.Context.encode_bound(n, nseg), dtype=torch.uint8, device="cuda")
        sbo = torch.zeros(nseg + 1, dtype=torch.int64, device="cuda")
        d = torch.empty(n, dtype=torch.int32, device="cuda")
        doff = torch.zeros(nseg + 1, dtype=torch.int64, device="cuda")
        def one():
            ctx.encode(sb, o, sbo, mode=mode)
            ctx.decode(o, sbo, nseg, n, d, doff)

        one()
        ctx.sync()
        assert torch.equal(d, sb.ids[:n]), "level %d round trip differs" % L
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            one()
        torch.cuda.synchronize()
        us = (time.perf_counter() - t) * 1e6 / reps
        comp = int(sbo[-1].item())
        res.append({"level": int(L), "ids": n, "ratio": round(4.0 * n / comp, 3), "us": round(us, 1),
                    "GBps": round(4.0 * n / (us * 1e-6) / 1e9, 2),
                    "classes": {"bitmap": int(c[0]), "bitpack": int(c[1:34].sum()), "pfor": int(c[34])}})
    return res


def exchange_leg(ctx, P, torch, g, root, host, nseg, mode, reps=3):
    """The first root's traversal through the candidate exchange of the 2D
    BFS: per level, every owner's unfiltered candidates (nseg*nseg segments)
    are compressed, decompressed, merged and filtered by the receivers.  The
    exchanged volume, its compression and the time of each phase (stream
    events), the best of `reps` traversals; the levels are checked against a
    plain GPU BFS."""
    V = g.n_vertices
    bounds_h = np.concatenate([[host["seg_lo"][0]], host["seg_hi"][:nseg]]).astype(np.uint32)
    if nseg > 256:  # 256 equal owners (65,536 segments per level) at most
        import inputs
        nseg = 256
        bounds_h = inputs.bounds_equal(V, nseg)
    RR = nseg * nseg
    dg = P.DeviceGraph.from_host(g)
    i32 = dict(dtype=torch.int32, device="cuda")
    level, parent = torch.empty(V, **i32), torch.empty(V, **i32)
    fa, fb = torch.empty(V, **i32), torch.empty(V, **i32)
    la, lb = torch.zeros(1, **i32), torch.zeros(1, **i32)
    bws = ctx.bfs_workspace(dg)
    xws = ctx.exchange_workspace(dg, nseg)
    ctx.exchange_init(dg, nseg, xws)
    bounds = torch.from_numpy(bounds_h.view(np.int32)).cuda()
    cap = max(1, g.n_arcs)
    ids = torch.zeros(cap, **i32)
    seg_off = torch.zeros(RR + 1, dtype=torch.int64, device="cuda")
    seg_lo, seg_hi = torch.zeros(RR, **i32), torch.zeros(RR, **i32)
    seg_level = torch.zeros(RR, **i32)
    db = P.DeviceBatch(ids, seg_off, seg_lo, seg_hi, seg_level, max_ids=cap)
    bcap = P.Context.encode_bound(cap, RR)
    stream = torch.zeros(bcap, dtype=torch.uint8, device="cuda")
    sbo = torch.zeros(RR + 1, dtype=torch.int64, device="cuda")
    out = torch.zeros(cap, **i32)
    out_off = torch.zeros(RR + 1, dtype=torch.int64, device="cuda")

    def traversal():
        ctx.bfs_init(dg, root, level, parent, fa, la, bws)
        f, fn, nxt, nn = fa, la, fb, lb
        rows, L = [], 0
        while True:
            n = int(fn.item())
            if n == 0:
                break
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            seg_level.fill_(L)  # a feature of the learned selector
            ev[0].record()
            ctx.candidates(dg, f, fn, bounds, ids, seg_off, seg_lo, seg_hi, xws)
            ev[1].record()
            ctx.encode(db, stream, sbo, mode=mode, out_cap=bcap)
            ctx.decode(stream, sbo, RR, cap, out, out_off)
            ev[2].record()
            ctx.merge_filter(dg, L, out, out_off[RR:], level, nxt, nn, bws, xws)
            ev[3].record()
            torch.cuda.synchronize()
            rows.append(dict(level=L, frontier=n, candidates=int(seg_off[-1].item()),
                             bytes=int(sbo[-1].item()), us_candidates=ev[0].elapsed_time(ev[1]) * 1e3,
                             us_codec=ev[1].elapsed_time(ev[2]) * 1e3, us_merge=ev[2].elapsed_time(ev[3]) * 1e3))
            f, fn, nxt, nn = nxt, nn, f, fn
            L += 1
        return rows

    traversal()
    assert ctx.sync_status() == 0, "candidate exchange reported an error"
    got = level.clone()
    # the same levels from the plain BFS (filtered frontier, no exchange),
    # each level timed for comparison
    bfs_us = []
    for rep in range(reps):
        ctx.bfs_init(dg, root, level, parent, fa, la, bws)
        L, us = 0, []
        while int(la.item()):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.bfs_level(dg, L, fa, la, level, parent, fb, lb, bws)
            e1.record()
            torch.cuda.synchronize()
            us.append(e0.elapsed_time(e1) * 1e3)
            fa, fb, la, lb = fb, fa, lb, la
            L += 1
        if not bfs_us or sum(us) < sum(bfs_us):
            bfs_us = us
    assert torch.equal(got, level), "exchange traversal levels differ from the BFS"
    best = None
    for _ in range(reps):
        rows = traversal()
        t = sum(r["us_candidates"] + r["us_codec"] + r["us_merge"] for r in rows)
        if best is None or t < best[0]:
            best = (t, rows)
    rows = best[1]
    cand = sum(r["candidates"] for r in rows)
    comp = sum(r["bytes"] for r in rows)
    codec_us = sum(r["us_codec"] for r in rows)
    return {"owners": nseg, "segments": RR, "levels": len(rows),
            "frontier_ids": sum(r["frontier"] for r in rows), "candidate_ids": cand, "compressed_bytes": comp,
            "ratio": round(4.0 * cand / max(1, comp), 3),
            "ms_candidates": round(sum(r["us_candidates"] for r in rows) / 1e3, 4),
            "ms_codec": round(codec_us / 1e3, 4),
            "ms_merge_filter": round(sum(r["us_merge"] for r in rows) / 1e3, 4),
            "codec_GBps": round(4.0 * cand / max(1e-9, codec_us * 1e-6) / 1e9, 2),
            "ms_bfs_levels": round(sum(bfs_us) / 1e3, 4),
            "per_level": [{"level": r["level"], "frontier": r["frontier"], "candidates": r["candidates"],
                           "ratio": round(4.0 * r["candidates"] / max(1, r["bytes"]), 3),
                           "us_candidates": round(r["us_candidates"], 1), "us_codec": round(r["us_codec"], 1),
                           "us_merge": round(r["us_merge"], 1), "us_bfs_level": round(u, 1)}
                          for r, u in zip(rows, bfs_us)]}


def bitmap_leg(ctx, P, torch, g, root, owners=(16, 64), reps=3):
    """The bitmap codec on the first root's traversal: at every level the
    frontier and the visited list as bitmaps, split into `owners` equal word
    ranges (one owner's share each), compressed and decompressed on the GPU
    and checked word for word; the final visited bitmap is the one a
    predecessor reduction would exchange.  Ratio = raw bitmap bytes over
    compressed bytes; GB/s of raw bitmap bytes over encode + decode (stream
    events, best of `reps`)."""
    V = g.n_vertices
    nw = (V + 31) // 32
    dg = P.DeviceGraph.from_host(g)
    i32 = dict(dtype=torch.int32, device="cuda")
    level, parent = torch.empty(V, **i32), torch.empty(V, **i32)
    fa, fb = torch.empty(V, **i32), torch.empty(V, **i32)
    la, lb = torch.zeros(1, **i32), torch.zeros(1, **i32)
    ws = ctx.bfs_workspace(dg, key="bm_bfs")
    ctx.bfs_init(dg, root, level, parent, fa, la, ws)
    L = 0
    while int(la.item()):
        ctx.bfs_level(dg, L, fa, la, level, parent, fb, lb, ws)
        fa, fb, la, lb = fb, fa, lb, la
        L += 1
    depth = L - 1
    shifts = torch.arange(32, device="cuda", dtype=torch.int64)

    def pack(mask):
        m = torch.zeros(nw * 32, dtype=torch.int64, device="cuda")
        m[:V] = mask.to(torch.int64)
        w = (m.view(nw, 32) << shifts).sum(dim=1)
        return torch.where(w >= 1 << 31, w - (1 << 32), w).to(torch.int32).contiguous()

    res = {"levels": depth + 1}
    for R in owners:
        seg_w = torch.from_numpy(((np.arange(R + 1, dtype=np.uint64) * nw) // R).view(np.int64)).cuda()
        cap = P.Context.bitmap_encode_bound(nw, R)
        out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
        sbo = torch.zeros(R + 1, dtype=torch.int64, device="cuda")
        back = torch.empty(nw, **i32)
        boff = torch.zeros(R + 1, dtype=torch.int64, device="cuda")
        wse = ctx.workspace(P._lib.OP_BITMAP_ENCODE, nw, R, key="bm_e")
        wsd = ctx.workspace(P._lib.OP_BITMAP_DECODE, nw, R, key="bm_d")
        row = {}
        for kind in ("frontier", "visited"):
            raw, comp, us = 0, 0, 0.0
            for Lv in range(depth + 1):
                bits = pack(level == Lv) if kind == "frontier" else pack((level >= 0) & (level <= Lv))
                best = None
                for _ in range(reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    ctx.bitmap_encode(bits, seg_w, R, nw, out, sbo, ws=wse)
                    ctx.bitmap_decode(out, sbo, R, nw, back, boff, ws=wsd)
                    e1.record()
                    torch.cuda.synchronize()
                    t = e0.elapsed_time(e1) * 1e3
                    best = t if best is None else min(best, t)
                assert ctx.sync_status() == 0, "bitmap codec reported an error"
                assert torch.equal(back, bits), "bitmap round trip differs"
                raw += 4 * nw
                comp += int(sbo[-1].item())
                us += best
            row[kind] = {"raw_bytes": raw, "compressed_bytes": comp, "ratio": round(raw / max(1, comp), 3),
                         "GBps": round(raw / max(1e-9, us * 1e-6) / 1e9, 2)}
        row["final_visited_ratio"] = round(4 * nw / max(1, int(sbo[-1].item())), 3)
        res["owners_%d" % R] = row
    return res


def mall_cold(ctx, P, torch, b, buf, sbo, dec, doff, N, mode, steps):
    """Encode + decode with a 1 GiB scratch write before every step, so that
    nothing of the batch is left in the 256 MB MALL; only the codec is timed
    (stream events around it)."""
    scratch = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for i in range(steps):
        scratch.fill_(i)
        ev[i][0].record()
        ctx.encode(b, buf, sbo, mode=mode)
        ctx.decode(buf, sbo, b.nseg, N, dec, doff)
        ev[i][1].record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(z) for a, z in ev)
    med = ms[len(ms) // 2]
    return {"ms_per_step_median": round(med, 4), "value_GBps": round(4.0 * N / (med * 1e-3) / 1e9, 2)}


def ratio_per_level(sbo_h, host):
    """[level, IDs, compression ratio] over all segments of each BFS level
    (levels of the different roots pooled)."""
    sizes = np.diff(host["seg_off"].astype(np.int64))
    nbytes = np.diff(sbo_h.astype(np.int64))
    lev = host["seg_level"].astype(np.int64)
    out = []
    for L in np.unique(lev):
        k = lev == L
        n = int(sizes[k].sum())
        out.append([int(L), n, round(4.0 * n / max(1, int(nbytes[k].sum())), 3)])
    return out


def check_segments(out, sbo_h, b, host, mode, n_check=24, cls=None):
    """Sampled segments of the full-size batch: GPU bytes equal the oracle's
    encoding of that segment alone (segments are independent), with the
    GPU's own per-block choice when a trained selector made it."""
    import oracle
    ids = b.ids[:b.max_ids].cpu().numpy().view(np.uint32)
    R = b.nseg
    rng = np.random.default_rng(0)
    sizes = np.diff(host["seg_off"].astype(np.int64))
    big = np.argsort(sizes)[-4:]
    pick = np.unique(np.concatenate([big, rng.choice(R, min(R, n_check), replace=False)]))
    data = out[:int(sbo_h[-1])].cpu().numpy()
    blk0 = np.concatenate([[0], np.cumsum((sizes + 127) // 128)])
    for r in pick:
        s, e = int(host["seg_off"][r]), int(host["seg_off"][r + 1])
        ob = oracle.Batch(ids[s:e], [0, e - s], [host["seg_lo"][r]], [host["seg_hi"][r]],
                          [host["seg_level"][r]])
        if cls is None:
            want, _ = oracle.encode(ob, mode=mode)
        else:
            k0 = int(blk0[r])
            want, _ = oracle.encode(ob, classes=cls[k0:k0 + (e - s + 127) // 128])
        got = data[int(sbo_h[r]):int(sbo_h[r + 1])]
        assert np.array_equal(got, want), "segment %d differs from the oracle" % r


def cpu_baseline(b, host, seconds, mode):
    """The oracle's encode + decode on a bounded sample of the same batch,
    single thread on this host, scaled to GB/s of raw bytes.  With the trained
    selector, the oracle's own path: fp64 forward pass, resolve, encode."""
    import oracle
    from oracle import mlp
    theta = None
    if mode == 2:
        theta = np.load(os.path.join(ROOT, "paper_1704_00513_amd", "selector_weights.npy"),
                        allow_pickle=False).astype(np.float64)
    ids = b.ids[:b.max_ids].cpu().numpy().view(np.uint32)
    R = b.nseg
    order = np.random.default_rng(1).permutation(R)
    done_ids, t_used, segs = 0, 0.0, 0
    for r in order:
        s, e = int(host["seg_off"][r]), int(host["seg_off"][r + 1])
        if e == s:
            continue
        ob = oracle.Batch(ids[s:e], [0, e - s], [host["seg_lo"][r]], [host["seg_hi"][r]],
                          [host["seg_level"][r]])
        t = time.perf_counter()
        if theta is None:
            stream, sbo = oracle.encode(ob, mode=mode)
        else:
            pred = mlp.predict(theta, mlp.features_to_f64(oracle.features(ob)))
            stream, sbo = oracle.encode(ob, classes=oracle.resolve(ob, pred)[0])
        st, got, _ = oracle.decode(stream, sbo)
        t_used += time.perf_counter() - t
        assert st == 0
        done_ids += e - s
        segs += 1
        if t_used >= seconds:
            break
    return {"value": round(4.0 * done_ids / t_used / 1e9, 4), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d random segments (%d IDs, %.1f%% of the batch), encode+decode, %.1f s"
                      % (segs, done_ids, 100.0 * done_ids / max(1, b.max_ids), t_used),
            "cpu": cpu_model()}


def cpu_baseline_threads(b, host, seconds, mode):
    """The same oracle calls spread over every host core (one segment per
    task; the oracle's C code runs without the interpreter lock)."""
    import concurrent.futures as cf
    import oracle
    from oracle import mlp
    theta = None
    if mode == 2:
        theta = np.load(os.path.join(ROOT, "paper_1704_00513_amd", "selector_weights.npy"),
                        allow_pickle=False).astype(np.float64)
    ids = b.ids[:b.max_ids].cpu().numpy().view(np.uint32)
    T = max(1, len(os.sched_getaffinity(0)))
    order = [r for r in np.random.default_rng(1).permutation(b.nseg)
             if host["seg_off"][r + 1] > host["seg_off"][r]]

    def work(r):
        s, e = int(host["seg_off"][r]), int(host["seg_off"][r + 1])
        ob = oracle.Batch(ids[s:e], [0, e - s], [host["seg_lo"][r]], [host["seg_hi"][r]],
                          [host["seg_level"][r]])
        if theta is None:
            stream, sbo = oracle.encode(ob, mode=mode)
        else:
            pred = mlp.predict(theta, mlp.features_to_f64(oracle.features(ob)))
            stream, sbo = oracle.encode(ob, classes=oracle.resolve(ob, pred)[0])
        st, _, _ = oracle.decode(stream, sbo)
        assert st == 0
        return e - s

    done, segs = 0, 0
    t = time.perf_counter()
    with cf.ThreadPoolExecutor(T) as ex:
        for k in range(0, len(order), 4 * T):
            done += sum(ex.map(work, order[k:k + 4 * T]))
            segs += len(order[k:k + 4 * T])
            if time.perf_counter() - t >= seconds:
                break
    el = time.perf_counter() - t
    return {"value": round(4.0 * done / el / 1e9, 4), "unit": "GB/s", "cores": T, "kind": "oracle",
            "sample": "%d random segments (%d IDs), encode+decode, %.1f s" % (segs, done, el)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
