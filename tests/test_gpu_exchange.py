"""GPU parity of the candidate exchange (the compressed row exchange of the
2D BFS: every owner's unfiltered candidates, compressed, decompressed, merged
and filtered by the receivers) against the oracle: candidate batches equal,
their streams byte for byte, and a traversal driven only by the exchange
reaching the textbook BFS frontiers and levels."""
from types import SimpleNamespace

import numpy as np
import pytest

import inputs
import oracle

from gpu_util import to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _bounds(V, nseg):
    if nseg == 5:  # uneven owners, one of them empty
        return np.array([0, 7, V // 3, V // 3, V // 2 + 11, V], np.uint32)
    return inputs.bounds_equal(V, nseg)


def exchange_traversal(ctx, g, root, bounds):
    """The whole traversal through bfsc_candidates -> bfsc_encode ->
    bfsc_decode -> bfsc_merge_filter, each level checked against the oracle."""
    import paper_1704_00513_amd as P
    t = torch()
    V = g.n_vertices
    R = bounds.size - 1
    RR = R * R
    dg = P.DeviceGraph.from_host(g)
    olv, _, depth = oracle.bfs(g, root)
    level = t.empty(V, dtype=t.int32, device="cuda")
    parent = t.empty(V, dtype=t.int32, device="cuda")
    fa = t.empty(V, dtype=t.int32, device="cuda")
    fb = t.empty(V, dtype=t.int32, device="cuda")
    la = t.zeros(1, dtype=t.int32, device="cuda")
    lb = t.zeros(1, dtype=t.int32, device="cuda")
    bws = ctx.bfs_workspace(dg)
    ctx.bfs_init(dg, root, level, parent, fa, la, bws)
    xws = ctx.exchange_workspace(dg, R)
    ctx.exchange_init(dg, R, xws)
    bdev = to_dev(bounds, np.uint32, np.int32)
    cap = max(1, g.n_arcs)
    ids = t.zeros(cap, dtype=t.int32, device="cuda")
    seg_off = t.zeros(RR + 1, dtype=t.int64, device="cuda")
    seg_lo = t.zeros(RR, dtype=t.int32, device="cuda")
    seg_hi = t.zeros(RR, dtype=t.int32, device="cuda")
    L = 0
    while True:
        n = int(la.item())
        fr = fa[:n].cpu().numpy().view(np.uint32)
        np.testing.assert_array_equal(fr, oracle.frontier(olv, L))
        if n == 0:
            break
        print("exchange V=%d R=%d level=%d frontier=%d" % (V, R, L, n), flush=True)
        ctx.candidates(dg, fa, la, bdev, ids, seg_off, seg_lo, seg_hi, xws)
        assert ctx.sync_status() == 0
        want = oracle.candidates(g, fr, bounds, L)
        total = int(seg_off[-1].item())
        np.testing.assert_array_equal(seg_off.cpu().numpy().view(np.uint64), want.seg_off)
        np.testing.assert_array_equal(ids[:total].cpu().numpy().view(np.uint32), want.ids)
        np.testing.assert_array_equal(seg_lo.cpu().numpy().view(np.uint32), want.seg_lo)
        np.testing.assert_array_equal(seg_hi.cpu().numpy().view(np.uint32), want.seg_hi)
        # compress the exchanged segments, decompress them at the receivers
        lev = t.full((RR,), L, dtype=t.int32, device="cuda")
        db = P.DeviceBatch(ids, seg_off, seg_lo, seg_hi, lev, max_ids=max(total, 1))
        bcap = P.Context.encode_bound(max(total, 1), RR)
        stream = t.zeros(bcap + 64, dtype=t.uint8, device="cuda")
        sbo = t.zeros(RR + 1, dtype=t.int64, device="cuda")
        ctx.encode(db, stream, sbo, out_cap=bcap)
        assert ctx.sync_status() == 0
        sbo_h = sbo.cpu().numpy().view(np.uint64)
        want_stream, want_off = oracle.encode(want)
        np.testing.assert_array_equal(sbo_h, want_off)
        np.testing.assert_array_equal(stream[:int(sbo_h[-1])].cpu().numpy(), want_stream)
        out = t.zeros(max(total, 1), dtype=t.int32, device="cuda")
        out_off = t.zeros(RR + 1, dtype=t.int64, device="cuda")
        ctx.decode(stream, sbo, RR, max(total, 1), out, out_off)
        ctx.merge_filter(dg, L, out, out_off[RR:], level, fb, lb, bws, xws)
        assert ctx.sync_status() == 0
        fa, fb, la, lb = fb, fa, lb, la
        L += 1
        assert L <= depth + 1
    np.testing.assert_array_equal(level.cpu().numpy(), olv)


@pytest.mark.parametrize("kind,scale,seed,nseg", [(inputs.RMAT, 14, 1, 16), (inputs.RMAT, 16, 2, 5),
                                                  (inputs.UNIFORM, 14, 3, 8), (inputs.RMAT, 12, 4, 1),
                                                  (inputs.RMAT, 14, 7, 100), (inputs.RMAT, 16, 8, 200),
                                                  (inputs.UNIFORM, 16, 9, 333)])
def test_exchange_traversal_matches_bfs(ctx, kind, scale, seed, nseg):
    g = inputs.graph(kind, scale, 16, seed)
    root = int(inputs.roots(g, 1, seed)[0])
    exchange_traversal(ctx, g, root, _bounds(g.n_vertices, nseg))


def _induced(g, V):
    """The subgraph on vertices [0, V) (still symmetric, rows ascending)."""
    rp = np.asarray(g.row_ptr, np.int64)
    rows = [g.col_idx[rp[u]:rp[u + 1]] for u in range(V)]
    rows = [r[r < V] for r in rows]
    row_ptr = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.uint64)
    col_idx = np.concatenate(rows).astype(np.uint32)
    return SimpleNamespace(row_ptr=row_ptr, col_idx=col_idx, n_vertices=V, n_arcs=int(col_idx.size))


@pytest.mark.parametrize("V,nseg", [(4001, 3), (3000, 7)])
def test_exchange_vertex_count_not_a_multiple_of_32(ctx, V, nseg):
    g = _induced(inputs.graph(inputs.RMAT, 12, 16, 6), V)
    root = int(np.argmax(np.diff(g.row_ptr.astype(np.int64))))
    bounds = np.linspace(0, V, nseg + 1).astype(np.uint32)
    exchange_traversal(ctx, g, root, bounds)


def test_exchange_capacity_and_bounds_are_reported(ctx):
    """Too small an ID buffer reports BFSC_E_CAPACITY (and writes nothing past
    it); owners that do not cover [0, V) report BFSC_E_INVAL."""
    import paper_1704_00513_amd as P
    t = torch()
    g = inputs.graph(inputs.RMAT, 12, 16, 5)
    root = int(inputs.roots(g, 1, 5)[0])
    level, _, _ = oracle.bfs(g, root)
    L = int(np.argmax([oracle.frontier(level, k).size for k in range(int(level.max()) + 1)]))
    f = oracle.frontier(level, L)
    dg = P.DeviceGraph.from_host(g)
    fd = to_dev(f, np.uint32, np.int32)
    fl = to_dev(np.array([f.size], np.uint32), np.uint32, np.int32)
    R = 4
    xws = ctx.exchange_workspace(dg, R)
    ctx.exchange_init(dg, R, xws)
    bounds = inputs.bounds_equal(g.n_vertices, R)
    want = oracle.candidates(g, f, bounds, L)
    assert want.n_ids > 100
    cap = want.n_ids // 2
    ids = t.full((cap + 64,), -1, dtype=t.int32, device="cuda")
    so = t.zeros(R * R + 1, dtype=t.int64, device="cuda")
    lo = t.zeros(R * R, dtype=t.int32, device="cuda")
    hi = t.zeros(R * R, dtype=t.int32, device="cuda")
    ctx.candidates(dg, fd, fl, to_dev(bounds, np.uint32, np.int32), ids, so, lo, hi, xws, cap=cap)
    assert ctx.sync_status() == 2
    tail = ids[cap:].cpu().numpy()
    assert (tail == -1).all()
    np.testing.assert_array_equal(ids[:cap].cpu().numpy().view(np.uint32), want.ids[:cap])
    # owners that do not start at 0 (room for every candidate, so that only
    # the bounds are wrong)
    bad = bounds.copy()
    bad[0] = 3
    ids2 = t.zeros(2 * want.n_ids, dtype=t.int32, device="cuda")
    ctx.candidates(dg, fd, fl, to_dev(bad, np.uint32, np.int32), ids2, so, lo, hi, xws)
    assert ctx.sync_status() == 1
    # still usable afterwards
    ids2 = t.zeros(want.n_ids, dtype=t.int32, device="cuda")
    ctx.candidates(dg, fd, fl, to_dev(bounds, np.uint32, np.int32), ids2, so, lo, hi, xws)
    assert ctx.sync_status() == 0
    np.testing.assert_array_equal(ids2.cpu().numpy().view(np.uint32), want.ids)
