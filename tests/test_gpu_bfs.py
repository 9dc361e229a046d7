"""GPU parity of the BFS level and the partitioner against the oracle: levels
and frontiers exact, parents valid under the oracle checker."""
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


def gpu_bfs(ctx, g, root):
    """Runs the whole traversal level by level; returns level, parent and the
    frontier list."""
    import paper_1704_00513_amd as P
    t = torch()
    dg = P.DeviceGraph.from_host(g)
    V = g.n_vertices
    level = t.empty(V, dtype=t.int32, device="cuda")
    parent = t.empty(V, dtype=t.int32, device="cuda")
    fa = t.empty(V, dtype=t.int32, device="cuda")
    fb = t.empty(V, dtype=t.int32, device="cuda")
    la = t.zeros(1, dtype=t.int32, device="cuda")
    lb = t.zeros(1, dtype=t.int32, device="cuda")
    ws = ctx.bfs_workspace(dg)
    ctx.bfs_init(dg, root, level, parent, fa, la, ws)
    fronts = []
    L = 0
    while True:
        n = int(la.item())
        if n == 0:
            break
        fronts.append(fa[:n].cpu().numpy().view(np.uint32).copy())
        ctx.bfs_level(dg, L, fa, la, level, parent, fb, lb, ws)
        fa, fb, la, lb = fb, fa, lb, la
        L += 1
        assert L <= V
    assert ctx.sync_status() == 0
    return level.cpu().numpy(), parent.cpu().numpy(), fronts


@pytest.mark.parametrize("kind,scale,seed", [(inputs.RMAT, 10, 1), (inputs.RMAT, 16, 1),
                                             (inputs.UNIFORM, 14, 2), (inputs.RMAT, 18, 3)])
def test_levels_frontiers_and_parents(ctx, kind, scale, seed):
    g = inputs.graph(kind, scale, 16, seed)
    for root in inputs.roots(g, 2, seed):
        print("bfs kind=%d scale=%d seed=%d root=%d" % (kind, scale, seed, root), flush=True)
        lv, par, fronts = gpu_bfs(ctx, g, int(root))
        olv, opar, depth = oracle.bfs(g, int(root))
        np.testing.assert_array_equal(lv, olv)
        assert oracle.bfs_check(g, int(root), lv, par) == 0
        assert len(fronts) == depth + 1
        for L, f in enumerate(fronts):
            np.testing.assert_array_equal(f, oracle.frontier(olv, L))


@pytest.mark.parametrize("alpha,beta", [(14.0, 24.0), (1e9, 1e9), (2.0, 0.5)])
@pytest.mark.parametrize("kind,scale,seed", [(inputs.RMAT, 10, 1), (inputs.RMAT, 16, 1),
                                             (inputs.UNIFORM, 14, 2), (inputs.RMAT, 18, 3)])
def test_direction_optimizing_levels(ctx, kind, scale, seed, alpha, beta):
    """Bottom-up levels (Beamer's switching rule; alpha = beta = 1e9 runs
    every level bottom-up): the same levels and frontiers as the textbook BFS,
    parents valid under the oracle checker."""
    g = inputs.graph(kind, scale, 16, seed)
    ctx.bfs_set_direction(alpha, beta)
    try:
        for root in inputs.roots(g, 2, seed):
            print("bfs-do kind=%d scale=%d seed=%d root=%d alpha=%g beta=%g" % (kind, scale, seed, root, alpha, beta),
                  flush=True)
            lv, par, fronts = gpu_bfs(ctx, g, int(root))
            olv, opar, depth = oracle.bfs(g, int(root))
            np.testing.assert_array_equal(lv, olv)
            assert oracle.bfs_check(g, int(root), lv, par) == 0
            assert len(fronts) == depth + 1
            for L, f in enumerate(fronts):
                np.testing.assert_array_equal(f, oracle.frontier(olv, L))
    finally:
        ctx.bfs_set_direction(0.0, 0.0)


@pytest.mark.parametrize("alpha,beta", [(0.0, 0.0), (1e9, 1e9)])
def test_vertex_count_not_a_multiple_of_64(ctx, alpha, beta):
    """The subgraph on the first 3001 vertices of an R-MAT graph: the last
    bitmap words are partial."""
    from types import SimpleNamespace
    g0 = inputs.graph(inputs.RMAT, 12, 16, 6)
    V = 3001
    rp = np.asarray(g0.row_ptr, np.int64)
    rows = [g0.col_idx[rp[u]:rp[u + 1]] for u in range(V)]
    rows = [r[r < V] for r in rows]
    row_ptr = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.uint64)
    col_idx = np.concatenate(rows).astype(np.uint32)
    g = SimpleNamespace(row_ptr=row_ptr, col_idx=col_idx, n_vertices=V, n_arcs=int(col_idx.size))
    root = int(np.argmax(np.diff(row_ptr.astype(np.int64))))
    ctx.bfs_set_direction(alpha, beta)
    try:
        print("bfs ragged V=%d alpha=%g" % (V, alpha), flush=True)
        lv, par, fronts = gpu_bfs(ctx, g, root)
    finally:
        ctx.bfs_set_direction(0.0, 0.0)
    olv, _, depth = oracle.bfs(g, root)
    np.testing.assert_array_equal(lv, olv)
    assert oracle.bfs_check(g, root, lv, par) == 0
    for L, f in enumerate(fronts):
        np.testing.assert_array_equal(f, oracle.frontier(olv, L))


def test_direction_arguments_are_checked(ctx):
    for alpha, beta in ((-1.0, 24.0), (14.0, 0.0), (float("nan"), 1.0)):
        with pytest.raises(Exception):
            ctx.bfs_set_direction(alpha, beta)
    ctx.bfs_set_direction(0.0, 0.0)


def test_isolated_root_has_one_level(ctx):
    # a vertex of degree zero: the traversal stops after the root
    g = inputs.graph(inputs.RMAT, 12, 16, 1)
    iso = int(np.flatnonzero(np.diff(g.row_ptr) == 0)[0])
    lv, par, fronts = gpu_bfs(ctx, g, iso)
    assert len(fronts) == 1 and list(fronts[0]) == [iso]
    assert (lv >= 0).sum() == 1


def test_partition_matches_oracle(ctx):
    t = torch()
    rng = np.random.default_rng(2)
    for trial in range(10):
        ids = inputs.random_sorted(int(rng.integers(0, 20000)), 1 << 20, trial)
        R = int(rng.choice([1, 16, 256, 1024]))
        bounds = inputs.bounds_equal(1 << 20, R) if trial % 2 else inputs.bounds_zipf(1 << 20, R, trial)[0]
        print("partition trial=%d n=%d R=%d" % (trial, ids.size, R), flush=True)
        seg_off = t.zeros(R + 1, dtype=t.int64, device="cuda")
        ctx.partition(to_dev(ids, np.uint32, np.int32), to_dev([ids.size], np.uint32, np.int32),
                      to_dev(bounds, np.uint32, np.int32), seg_off)
        got = seg_off.cpu().numpy().view(np.uint64)
        np.testing.assert_array_equal(got, oracle.partition(ids, bounds))
