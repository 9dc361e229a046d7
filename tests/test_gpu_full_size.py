"""Parity at full size, with the frontiers made by the direction-optimizing
BFS as the benchmark makes them: R-MAT s22 (edge factor 16, seed 1), 8 roots,
every level split into 16 equal vertex ranges, exhaustive choice, default
launch configuration (the benchmark's timed workload); and R-MAT s24, 8
roots, 256 Zipf-sized ranges per level, launch shapes from the autotuner.  The oracle checks what it can compute piece by piece: the first
root's levels and parents, and sampled segments byte for byte (segments are
independent); the full round trip and the offsets are checked at full size.
The uniform s24 and the s26 workloads are checked the same way by the
benchmark itself before it times them (sampled segments, full round trip),
which keeps this file near a minute."""
import numpy as np
import pytest

import inputs
import oracle

from gpu_util import torch

pytestmark = pytest.mark.gpu

ROOTS = 8
CASES = [(inputs.RMAT, 22, 16, False), (inputs.RMAT, 24, 256, True)]


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module", params=CASES, ids=["rmat-s22-equal16", "rmat-s24-zipf256"])
def full(ctx, request):
    import paper_1704_00513_amd as P
    t = torch()
    kind, scale, NSEG, zipf = request.param
    print("full-size batch: kind=%d s%d, %d roots, %d segments per level" % (kind, scale, ROOTS, NSEG), flush=True)
    g = inputs.graph(kind, scale, 16, 1, cache=False)
    roots = inputs.roots(g, ROOTS, 1)
    V = g.n_vertices
    dg = P.DeviceGraph.from_host(g)
    bounds_h = inputs.bounds_zipf(V, NSEG, 1)[0] if zipf else inputs.bounds_equal(V, NSEG)
    bounds = t.from_numpy(bounds_h.view(np.int32)).cuda()
    i32 = dict(dtype=t.int32, device="cuda")
    all_ids = t.empty(V * (ROOTS + 1), **i32)
    level, parent = t.empty(V, **i32), t.empty(V, **i32)
    la, lb = t.zeros(1, **i32), t.zeros(1, **i32)
    seg_off_l = t.zeros(NSEG + 1, dtype=t.int64, device="cuda")
    ws = ctx.bfs_workspace(dg, key="full")
    ctx.bfs_set_direction(14.0, 24.0)
    offs, levs, base, root0 = [np.zeros(1, np.uint64)], [], 0, None
    try:
        for k, root in enumerate(roots):
            front = all_ids[base:]
            ctx.bfs_init(dg, int(root), level, parent, front, la, ws)
            L = 0
            while True:
                n = int(la.item())
                if n == 0:
                    break
                ctx.partition(front, la, bounds, seg_off_l)
                offs.append(seg_off_l.cpu().numpy().view(np.uint64)[1:] + np.uint64(base))
                levs.append(np.full(NSEG, L, np.int32))
                nxt = all_ids[base + n:]
                ctx.bfs_level(dg, L, front, la, level, parent, nxt, lb, ws)
                base += n
                front = nxt
                la, lb = lb, la
                L += 1
            if k == 0:
                root0 = (int(root), level.cpu().numpy(), parent.cpu().numpy())
    finally:
        ctx.bfs_set_direction(0.0, 0.0)
    assert ctx.sync_status() == 0
    seg_off = np.concatenate(offs)
    nlev = len(levs)
    lo, hi = np.tile(bounds_h[:-1], nlev), np.tile(bounds_h[1:], nlev)
    b = P.DeviceBatch(all_ids[:base], t.from_numpy(seg_off.view(np.int64)).cuda(),
                      t.from_numpy(lo.view(np.int32)).cuda(), t.from_numpy(hi.view(np.int32)).cuda(),
                      t.from_numpy(np.concatenate(levs)).cuda(), max_ids=base)
    yield dict(g=g, b=b, seg_off=seg_off, lo=lo, hi=hi, lev=np.concatenate(levs), n=base, root0=root0,
               autotune=zipf, scale=scale)
    del b, all_ids, dg


def test_full_size_first_root_levels_and_parents(full):
    if full["scale"] > 22:
        pytest.skip("the oracle BFS and its checker take about two minutes at s24; "
                    "levels and parents are checked at s22 and below")
    root, lv, par = full["root0"]
    print("full-size BFS check root=%d" % root, flush=True)
    olv, _, _ = oracle.bfs(full["g"], root)
    np.testing.assert_array_equal(lv, olv)
    assert oracle.bfs_check(full["g"], root, lv, par) == 0


def test_full_size_round_trip_and_sampled_segments(ctx, full):
    import paper_1704_00513_amd as P
    t = torch()
    b, N = full["b"], full["n"]
    R = b.nseg
    before = ctx.get_tune()
    if full["autotune"]:
        print("full-size autotune:", ctx.autotune(b), flush=True)
    print("full-size encode/decode: %d IDs in %d segments" % (N, R), flush=True)
    try:
        _round_trip_and_samples(ctx, full, P, t, b, N, R)
    finally:
        ctx.set_tune(**before)


def _round_trip_and_samples(ctx, full, P, t, b, N, R):
    cap = P.Context.encode_bound(N, R)
    out = t.zeros(cap, dtype=t.uint8, device="cuda")
    sbo = t.zeros(R + 1, dtype=t.int64, device="cuda")
    ctx.encode(b, out, sbo, mode=P.SEL_EXHAUSTIVE)
    assert ctx.sync_status() == 0
    dec = t.empty(N, dtype=t.int32, device="cuda")
    doff = t.zeros(R + 1, dtype=t.int64, device="cuda")
    ctx.decode(out, sbo, R, N, dec, doff)
    assert ctx.sync_status() == 0
    assert t.equal(dec, b.ids[:N])
    np.testing.assert_array_equal(doff.cpu().numpy().view(np.uint64), full["seg_off"])
    sbo_h = sbo.cpu().numpy().view(np.uint64)
    assert np.all(np.diff(sbo_h.astype(np.int64)) >= 16) and int(sbo_h[-1]) <= cap
    # sampled segments: the four largest and 24 random ones, byte for byte
    ids = b.ids[:N].cpu().numpy().view(np.uint32)
    data = out[:int(sbo_h[-1])].cpu().numpy()
    sizes = np.diff(full["seg_off"].astype(np.int64))
    pick = np.unique(np.concatenate([np.argsort(sizes)[-4:],
                                     np.random.default_rng(5).choice(R, 24, replace=False)]))
    for r in pick:
        s, e = int(full["seg_off"][r]), int(full["seg_off"][r + 1])
        ob = oracle.Batch(ids[s:e], [0, e - s], [full["lo"][r]], [full["hi"][r]], [full["lev"][r]])
        want, _ = oracle.encode(ob)
        np.testing.assert_array_equal(data[int(sbo_h[r]):int(sbo_h[r + 1])], want, err_msg="segment %d" % r)
