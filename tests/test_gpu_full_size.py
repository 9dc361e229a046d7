"""Parity at full size, with the frontiers made by the direction-optimizing
BFS as the benchmark makes them: R-MAT s22 (edge factor 16, seed 1), 8 roots,
every level split into 16 equal vertex ranges, exhaustive choice, default
launch configuration; R-MAT s24, 8 roots, 256 Zipf-sized ranges per level,
launch shapes from the autotuner; and R-MAT s24, 8 roots, 1024 Zipf-sized
ranges with the trained selector fused into the pack pass (the benchmark's
timed choice).  The oracle checks what it can compute piece by piece: the
first root's levels (the oracle BFS) and parents (a vectorised check of the
parent rules), and sampled segments byte for byte (segments are
independent); the full round trip and the offsets are checked at full size.
The uniform s24 and the s26 workloads are checked the same way by the
benchmark itself before it times them (sampled segments, full round trip).
"""
import numpy as np
import pytest

import inputs
import oracle

from gpu_util import torch

pytestmark = pytest.mark.gpu

ROOTS = 8
CASES = [(inputs.RMAT, 22, 16, False), (inputs.RMAT, 24, 256, True), (inputs.RMAT, 24, 1024, True)]


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module", params=CASES, ids=["rmat-s22-equal16", "rmat-s24-zipf256", "rmat-s24-zipf1024"])
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
               autotune=zipf and NSEG == 256, scale=scale, nseg=NSEG)
    del b, all_ids, dg


def parents_valid(g, root, level, parent):
    """The parent rules of a BFS tree, vectorised: the root is its own
    parent at level 0; unreached vertices have parent -1; a reached vertex's
    parent is one level closer and an arc joins them (found by a binary
    search of the vertex's own sorted adjacency row: the graph is
    undirected)."""
    V = g.n_vertices
    if level[root] != 0 or parent[root] != root:
        return False
    unreached = level < 0
    if not np.all(parent[unreached] == -1):
        return False
    v = np.flatnonzero(~unreached)
    v = v[v != root]
    p = parent[v].astype(np.int64)
    if np.any(p < 0) or np.any(p >= V) or np.any(level[p] != level[v] - 1):
        return False
    lo = g.row_ptr[v].astype(np.int64)
    hi = g.row_ptr[v + 1].astype(np.int64)
    col = g.col_idx
    while True:  # first index in [lo, hi) with col >= p
        act = lo < hi
        if not act.any():
            break
        mid = (lo + hi) >> 1
        c = col[np.minimum(mid, col.size - 1)].astype(np.int64)
        go = act & (c < p)
        lo = np.where(go, mid + 1, lo)
        hi = np.where(act & ~go, mid, hi)
    found = (lo < g.row_ptr[v + 1].astype(np.int64)) & (col[np.minimum(lo, col.size - 1)].astype(np.int64) == p)
    return bool(found.all())


def test_parent_check_catches_planted_mistakes():
    g = inputs.graph(inputs.RMAT, 12, 16, 1)
    root = int(inputs.roots(g, 1, 1)[0])
    lv, par, _ = oracle.bfs(g, root)
    assert parents_valid(g, root, lv, par)
    reached = np.flatnonzero((lv > 1))
    bad = par.copy()
    # a vertex one level closer that is not a neighbour
    v = int(reached[0])
    cand = np.flatnonzero(lv == lv[v] - 1)
    nbr = set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist())
    bad[v] = next(int(u) for u in cand if int(u) not in nbr)
    assert not parents_valid(g, root, lv, bad)
    bad = par.copy()
    bad[v] = v  # a vertex on its own level
    assert not parents_valid(g, root, lv, bad)


def test_full_size_first_root_levels_and_parents(full):
    root, lv, par = full["root0"]
    print("full-size BFS check s%d root=%d" % (full["scale"], root), flush=True)
    olv, _, _ = oracle.bfs(full["g"], root)
    np.testing.assert_array_equal(lv, olv)
    assert parents_valid(full["g"], root, lv, par)


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
    assert int(sbo_h[-1]) <= cap
    # the segment forms: empty 0 bytes, raw 4 n, compressed at least a header
    seg_n = np.diff(full["seg_off"].astype(np.int64))
    seg_b = np.diff(sbo_h.astype(np.int64))
    raw = (seg_n > 0) & (seg_n < oracle.RAW_BELOW)
    assert np.all(seg_b[seg_n == 0] == 0) and np.all(seg_b[raw] == 4 * seg_n[raw])
    assert np.all(seg_b[seg_n >= oracle.RAW_BELOW] >= 24)
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


def test_full_size_fused_learned_pass(ctx, full):
    """The trained selector inside the pack pass, on each full-size batch:
    the stream is the oracle's encoding (per sampled segment) of the class
    vector that the separate selection pass writes, and those classes are the
    oracle's resolved prediction wherever its top two logits are clearly
    apart."""
    import os
    import paper_1704_00513_amd as P
    from oracle import mlp
    t = torch()
    b, N = full["b"], full["n"]
    R = b.nseg
    theta = np.load(os.path.join(os.path.dirname(P.__file__), "selector_weights.npy"), allow_pickle=False)
    ctx.mlp_set_weights(theta)
    print("full-size learned: %d IDs in %d segments" % (N, R), flush=True)
    cap = P.Context.encode_bound(N, R)
    out = t.zeros(cap, dtype=t.uint8, device="cuda")
    sbo = t.zeros(R + 1, dtype=t.int64, device="cuda")
    ctx.encode(b, out, sbo, mode=P.SEL_LEARNED)
    assert ctx.sync_status() == 0
    cls = t.zeros(b.n_blocks_max, dtype=t.uint8, device="cuda")
    ctx.select(b, P.SEL_LEARNED, cls)
    dec = t.empty(N, dtype=t.int32, device="cuda")
    doff = t.zeros(R + 1, dtype=t.int64, device="cuda")
    ctx.decode(out, sbo, R, N, dec, doff)
    assert ctx.sync_status() == 0
    assert t.equal(dec, b.ids[:N])
    sbo_h = sbo.cpu().numpy().view(np.uint64)
    cls_h = cls.cpu().numpy()
    ids = b.ids[:N].cpu().numpy().view(np.uint32)
    data = out[:int(sbo_h[-1])].cpu().numpy()
    sizes = np.diff(full["seg_off"].astype(np.int64))
    blk0 = np.concatenate([[0], np.cumsum((sizes + 127) // 128)])
    pick = np.unique(np.concatenate([np.argsort(sizes)[-4:],
                                     np.random.default_rng(6).choice(R, 24, replace=False)]))
    th = theta.astype(np.float64)
    checked = 0
    for r in pick:
        s, e = int(full["seg_off"][r]), int(full["seg_off"][r + 1])
        ob = oracle.Batch(ids[s:e], [0, e - s], [full["lo"][r]], [full["hi"][r]], [full["lev"][r]])
        k0, k1 = int(blk0[r]), int(blk0[r + 1])
        want, _ = oracle.encode(ob, classes=cls_h[k0:k1])
        np.testing.assert_array_equal(data[int(sbo_h[r]):int(sbo_h[r + 1])], want, err_msg="segment %d" % r)
        if e - s >= oracle.RAW_BELOW:
            X = mlp.features_to_f64(oracle.features(ob))
            z, _ = mlp.forward(th, X)
            res, _ = oracle.resolve(ob, mlp.predict(th, X))
            top2 = np.sort(z, axis=1)[:, -2:]
            clear = (top2[:, 1] - top2[:, 0]) > 2e-3 * (1 + np.abs(top2[:, 1]))
            np.testing.assert_array_equal(cls_h[k0:k1][clear], res[clear], err_msg="segment %d" % r)
            checked += int(clear.sum())
    assert checked > 1000
