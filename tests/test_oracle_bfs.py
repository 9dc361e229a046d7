"""Pins of the oracle BFS, checker and partitioner: levels against a library
shortest-path routine, planted mistakes against every checker rule, and the
partition against numpy's searchsorted."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import inputs
import oracle


def scipy_levels(g, root):
    V = g.n_vertices
    A = sp.csr_matrix((np.ones(g.n_arcs, np.int8), g.col_idx.astype(np.int64),
                       g.row_ptr.astype(np.int64)), shape=(V, V))
    d = shortest_path(A, method="D", unweighted=True, indices=[int(root)])[0]
    return np.where(np.isinf(d), -1, d).astype(np.int64)


@pytest.mark.parametrize("kind,scale,seed", [(inputs.RMAT, 10, 1), (inputs.RMAT, 12, 2),
                                             (inputs.UNIFORM, 11, 3)])
def test_levels_equal_library_shortest_paths(kind, scale, seed):
    g = inputs.graph(kind, scale, 16, seed)
    for root in inputs.roots(g, 3, seed):
        level, parent, depth = oracle.bfs(g, root)
        np.testing.assert_array_equal(level.astype(np.int64), scipy_levels(g, root))
        assert depth == level.max()
        assert oracle.bfs_check(g, root, level, parent) == 0


def test_checker_catches_each_planted_mistake():
    g = inputs.graph(inputs.RMAT, 10, 16, 1)
    root = int(inputs.roots(g, 1, 1)[0])
    level, parent, depth = oracle.bfs(g, root)
    reached = np.flatnonzero(level > 0)
    v = int(reached[len(reached) // 2])

    bad = parent.copy(); bad[root] = -1
    assert oracle.bfs_check(g, root, level, bad) == 1
    unreached = np.flatnonzero(level < 0)
    if unreached.size:
        bad = parent.copy(); bad[unreached[0]] = root
        assert oracle.bfs_check(g, root, level, bad) == 2
    bad = parent.copy(); bad[v] = v  # parent not one level closer
    assert oracle.bfs_check(g, root, level, bad) == 3
    # a vertex one level closer that is not a neighbour
    nbrs = set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist())
    cand = [u for u in np.flatnonzero(level == level[v] - 1) if u not in nbrs]
    if cand:
        bad = parent.copy(); bad[v] = cand[0]
        assert oracle.bfs_check(g, root, level, bad) == 4
    badl = level.copy(); badl[v] += 2
    assert oracle.bfs_check(g, root, badl, parent) in (3, 5)
    # drop a reachable leaf: an arc then joins reached and unreached
    leaf = int(np.flatnonzero(level == depth)[0])
    badl = level.copy(); bad = parent.copy()
    badl[leaf] = -1; bad[leaf] = -1
    assert oracle.bfs_check(g, root, badl, bad) == 5


def test_frontiers_are_sorted_disjoint_and_cover_the_component():
    g = inputs.graph(inputs.RMAT, 12, 16, 1)
    root = int(inputs.roots(g, 1, 1)[0])
    level, parent, depth = oracle.bfs(g, root)
    fs = oracle.frontiers(level, depth)
    assert list(fs[0]) == [root]
    allv = np.concatenate(fs)
    assert allv.size == (level >= 0).sum() == np.unique(allv).size
    for L, f in enumerate(fs):
        assert f.size > 0 and np.all(np.diff(f.astype(np.int64)) > 0)
        assert np.all(level[f] == L)


def test_partition_matches_searchsorted():
    rng = np.random.default_rng(1)
    for t in range(20):
        ids = inputs.random_sorted(int(rng.integers(0, 5000)), 1 << 16, t)
        R = int(rng.integers(1, 40))
        bounds = np.sort(rng.integers(0, 1 << 16, R + 1)).astype(np.uint32)
        bounds[0], bounds[-1] = 0, 1 << 16
        off = oracle.partition(ids, bounds)
        want = np.searchsorted(ids, bounds, side="left")
        want[-1] = ids.size
        np.testing.assert_array_equal(off, want.astype(np.uint64))


def test_batch_from_frontier_concatenation_is_the_frontier():
    ids = inputs.random_sorted(10000, 1 << 20, 4)
    bounds, _ = inputs.bounds_zipf(1 << 20, 64, 4)
    b = oracle.batch_from_frontier(ids, bounds, 3)
    np.testing.assert_array_equal(b.ids, ids)
    for r in range(b.nseg):
        seg = ids[int(b.seg_off[r]):int(b.seg_off[r + 1])]
        assert np.all(seg >= bounds[r]) and np.all(seg < bounds[r + 1])


def test_config1_pipeline_round_trips_every_level():
    # R-MAT scale 16, edge factor 16, seed 1, one seeded root, each level as one
    # segment over [0, V), plain bit-packing at the minimal width
    g = inputs.graph(inputs.RMAT, 16, 16, 1)
    root = int(inputs.roots(g, 1, 1)[0])
    level, parent, depth = oracle.bfs(g, root)
    assert oracle.bfs_check(g, root, level, parent) == 0
    for L in range(depth + 1):
        f = oracle.frontier(level, L)
        b = oracle.batch_from_frontier(f, np.array([0, g.n_vertices], np.uint32), L)
        stream, sbo = oracle.encode(b, mode=oracle.PLAIN_BP)
        st, out, _ = oracle.decode(stream, sbo)
        assert st == oracle.ST_OK and np.array_equal(out, f)
        cls = oracle.select(b, oracle.PLAIN_BP)
        assert np.all((cls >= 1) & (cls <= 33))
