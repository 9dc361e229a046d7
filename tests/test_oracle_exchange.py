"""Pins of the candidate-exchange oracle (the compressed row exchange of the
2D BFS: unfiltered candidates per owner, then the receiver's merge and
visited filter) against the textbook BFS and brute force."""
import numpy as np

import inputs
import oracle


def _graph():
    return inputs.graph(inputs.RMAT, 14, 16, 3)


def _neighbours(g, vs):
    rp = np.asarray(g.row_ptr, np.int64)
    out = set()
    for u in vs:
        out.update(int(w) for w in g.col_idx[rp[u]:rp[u + 1]])
    return out


def test_merge_filter_of_candidates_is_the_next_frontier():
    """For every level: the union of all owners' unfiltered candidates, less
    the visited vertices, is exactly the textbook BFS frontier L+1, with level
    L+1 -- for one owner and for 16 and 5 uneven ones."""
    g = _graph()
    root = int(inputs.roots(g, 1, 1)[0])
    level, _, depth = oracle.bfs(g, root)
    for bounds in (np.array([0, g.n_vertices], np.uint32), inputs.bounds_equal(g.n_vertices, 16),
                   np.array([0, 7, 1000, 1001, 9000, g.n_vertices], np.uint32)):
        lv = np.full(g.n_vertices, -1, np.int32)
        lv[root] = 0
        for L in range(depth + 1):
            f = oracle.frontier(level, L)
            b = oracle.candidates(g, f, bounds, L)
            nxt, lv = oracle.merge_filter(b.ids, lv, L)
            np.testing.assert_array_equal(nxt, oracle.frontier(level, L + 1))
        np.testing.assert_array_equal(lv, level)


def test_candidate_segments_are_the_neighbour_sets():
    """Segment p*R + d holds, sorted and once each, the neighbours in owner d's
    range of the frontier vertices owner p holds (brute force over Python
    sets); a vertex reached by several owners is counted once per owner."""
    g = _graph()
    root = int(inputs.roots(g, 1, 2)[0])
    level, _, depth = oracle.bfs(g, root)
    bounds = inputs.bounds_equal(g.n_vertices, 6)
    R = bounds.size - 1
    L = int(np.argmax([oracle.frontier(level, k).size for k in range(depth + 1)]))
    f = oracle.frontier(level, L)
    b = oracle.candidates(g, f, bounds, L)
    assert b.nseg == R * R
    union = set()
    total = 0
    for p in range(R):
        fp = [int(u) for u in f if bounds[p] <= u < bounds[p + 1]]
        tp = _neighbours(g, fp)
        total += len(tp)
        union |= tp
        for d in range(R):
            s = b.ids[int(b.seg_off[p * R + d]):int(b.seg_off[p * R + d + 1])]
            want = sorted(w for w in tp if bounds[d] <= w < bounds[d + 1])
            assert s.tolist() == want
            assert b.seg_lo[p * R + d] == bounds[d] and b.seg_hi[p * R + d] == bounds[d + 1]
    assert b.n_ids == total >= len(union) == len(_neighbours(g, f.tolist()))


def test_candidates_on_a_small_graph_by_hand():
    """Path 0-1-2-3 plus the edge 1-3, frontier {1, 3}, owners [0, 2) and [2, 4):
    owner 0 (vertex 1) reaches {0, 2, 3}, owner 1 (vertex 3) reaches {1, 2}."""
    class G:
        n_vertices = 4
        row_ptr = np.array([0, 1, 4, 6, 8], np.uint64)
        col_idx = np.array([1, 0, 2, 3, 1, 3, 1, 2], np.uint32)
    b = oracle.candidates(G, np.array([1, 3], np.uint32), np.array([0, 2, 4], np.uint32), 1)
    assert b.ids.tolist() == [0, 2, 3, 1, 2]
    assert b.seg_off.tolist() == [0, 1, 3, 4, 5]
    lv = np.array([-1, 1, 0, 1], np.int32)
    nxt, lv = oracle.merge_filter(b.ids, lv, 1)
    assert nxt.tolist() == [0] and lv.tolist() == [2, 1, 0, 1]
