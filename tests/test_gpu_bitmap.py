"""GPU parity of the bitmap codec (one owner's share of a vertex bitmap)
against the CPU oracle through the C-ABI: byte-exact streams and offsets,
exact words, the same accept / reject decision on damaged streams."""
import numpy as np
import pytest

import inputs
import oracle

from gpu_util import to_dev, torch
from test_oracle_bitmap import random_bitmap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


def log(msg):
    print(msg, flush=True)


def gpu_bm_encode(ctx, words, seg_w, out_cap=None):
    import paper_1704_00513_amd as P
    t = torch()
    nseg = seg_w.size - 1
    max_words = int(seg_w[-1])
    cap = P.Context.bitmap_encode_bound(max_words, nseg) if out_cap is None else out_cap
    out = t.zeros(max(4, cap), dtype=t.uint8, device="cuda")
    sbo = t.zeros(nseg + 1, dtype=t.int64, device="cuda")
    ctx.bitmap_encode(to_dev(words, np.uint32, np.int32), to_dev(seg_w, np.uint64, np.int64), nseg, max_words,
                      out, sbo, out_cap=cap)
    st = ctx.sync_status()
    sbo_h = sbo.cpu().numpy().view(np.uint64)
    n = int(sbo_h[-1]) if st == 0 else 0
    return st, out[:n].cpu().numpy(), sbo_h


def gpu_bm_decode(ctx, stream, sbo, max_words, out_cap=None):
    t = torch()
    nseg = sbo.size - 1
    data = to_dev(np.concatenate([stream, np.zeros(4, np.uint8)]), np.uint8, np.uint8)
    cap = max_words if out_cap is None else out_cap
    out = t.zeros(max(1, cap), dtype=t.int32, device="cuda")
    off = t.zeros(nseg + 1, dtype=t.int64, device="cuda")
    ctx.bitmap_decode(data, to_dev(sbo, np.uint64, np.int64), nseg, max_words, out, off, out_cap=cap)
    st = ctx.sync_status()
    off_h = off.cpu().numpy().view(np.uint64)
    n = int(off_h[-1]) if st == 0 else 0
    return st, out[:n].cpu().numpy().view(np.uint32), off_h


def bfs_bitmaps(scale, nseg, seed=1):
    """Visited and frontier bitmaps of an R-MAT BFS (oracle levels) at every
    level, each split into nseg owners (word ranges of equal size)."""
    g = inputs.graph(inputs.RMAT, scale, 16, seed)
    level, _, depth = oracle.bfs(g, int(inputs.roots(g, 1, seed)[0]))
    V = g.n_vertices
    nw = (V + 31) // 32
    seg_w = (np.arange(nseg + 1, dtype=np.uint64) * nw) // nseg
    out = []
    for L in range(depth + 1):
        front = np.zeros(nw * 32, bool)
        front[:V] = level == L
        vis = np.zeros(nw * 32, bool)
        vis[:V] = (level >= 0) & (level <= L)
        out.append(("s%d-L%d-frontier" % (scale, L), words_of(front), seg_w))
        out.append(("s%d-L%d-visited" % (scale, L), words_of(vis), seg_w))
    return out


def words_of(bits):
    b = np.asarray(bits, bool).reshape(-1, 32)
    return (b.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)


def synthetic_cases():
    out = []
    for dens in (0.0, 0.001, 0.02, 0.3, 0.5, 0.9, 0.995, 1.0):
        w = random_bitmap(1500, dens, int(dens * 997) + 3)
        out.append(("dens%g" % dens, w, np.array([0, 1, 129, 129, 256, 900, 1500], np.uint64)))
    w = random_bitmap(9000, 0.2, 9, runs=True)
    out.append(("runs", w, np.array([0, 4000, 4001, 9000], np.uint64)))
    # many small segments, every size from 0 to 40 words
    sizes = np.arange(41)
    seg_w = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    out.append(("small", random_bitmap(int(seg_w[-1]), 0.05, 4, runs=True), seg_w))
    # more segments than one plan workgroup takes (1,024), empty ones among them
    sizes = np.random.default_rng(21).integers(0, 300, 2500)
    sizes[::7] = 0
    seg_w = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    out.append(("many", random_bitmap(int(seg_w[-1]), 0.1, 21, runs=True), seg_w))
    return out


def check_case(ctx, name, words, seg_w):
    log("bitmap case=%s words=%d segments=%d" % (name, int(seg_w[-1]), seg_w.size - 1))
    want, want_sbo = oracle.bmc_encode(words, seg_w)
    st, got, sbo = gpu_bm_encode(ctx, words, seg_w)
    assert st == 0, name
    np.testing.assert_array_equal(sbo, want_sbo, err_msg=name)
    np.testing.assert_array_equal(got, want, err_msg=name)
    st, back, off = gpu_bm_decode(ctx, got, sbo, int(seg_w[-1]))
    assert st == 0, name
    np.testing.assert_array_equal(back, words[int(seg_w[0]):int(seg_w[-1])], err_msg=name)
    np.testing.assert_array_equal(off, seg_w - seg_w[0], err_msg=name)


@pytest.mark.parametrize("case", synthetic_cases(), ids=lambda c: c[0])
def test_synthetic_bitmaps_byte_exact(ctx, case):
    check_case(ctx, *case)


@pytest.mark.parametrize("scale,nseg", [(14, 16), (16, 16), (16, 64)])
def test_bfs_bitmaps_byte_exact(ctx, scale, nseg):
    for name, words, seg_w in bfs_bitmaps(scale, nseg):
        check_case(ctx, name + "-R%d" % nseg, words, seg_w)


def test_damaged_streams_agree_with_oracle(ctx):
    rng = np.random.default_rng(12)
    for name, words, seg_w in synthetic_cases()[3:5] + [synthetic_cases()[8]]:
        stream, sbo = oracle.bmc_encode(words, seg_w)
        log("bitmap damage case=%s bytes=%d" % (name, stream.size))
        for trial in range(80):
            s = stream.copy()
            for _ in range(int(rng.integers(1, 3))):
                pos = int(rng.integers(0, s.size))
                s[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
            want_st, want, _ = oracle.bmc_decode(s, sbo, out_cap=int(seg_w[-1]))
            st, got, _ = gpu_bm_decode(ctx, s, sbo, int(seg_w[-1]))
            assert (st == 0) == (want_st == 0), (name, trial, st, want_st)
            if st == 0:
                np.testing.assert_array_equal(got, want)


def test_capacity_is_reported(ctx):
    words = random_bitmap(2000, 0.4, 5)
    seg_w = np.array([0, 1000, 2000], np.uint64)
    st, _, _ = gpu_bm_encode(ctx, words, seg_w, out_cap=100)
    assert st != 0
    stream, sbo = oracle.bmc_encode(words, seg_w)
    st, _, _ = gpu_bm_decode(ctx, stream, sbo, 2000, out_cap=1999)
    assert st != 0
    st, back, _ = gpu_bm_decode(ctx, stream, sbo, 2000)
    assert st == 0 and np.array_equal(back, words)
