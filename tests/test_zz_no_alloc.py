"""bfsc_decode_noalloc (the decoder with the library's fixed scratch array
instead of a workspace) against bfsc_decode on the same streams: IDs and
offsets bit-exact, on two calls in a row, the second with a smaller input,
and both equal to the oracle's decode."""
import numpy as np
import pytest

import inputs
import oracle

from gpu_util import gpu_encode, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


def log(msg):
    print(msg, flush=True)


def both_decodes(ctx, stream, sbo, max_ids):
    """Decodes one stream with bfsc_decode and with bfsc_decode_noalloc into
    separate buffers; returns both (status, ids, offsets)."""
    import torch
    nseg = sbo.size - 1
    data = to_dev(np.concatenate([stream, np.zeros(4, np.uint8)]), np.uint8, np.uint8)
    sbo_d = to_dev(sbo, np.uint64, np.int64)
    res = []
    for noalloc in (False, True):
        out = torch.full((max(1, max_ids),), -7, dtype=torch.int32, device="cuda")
        off = torch.full((nseg + 1,), -7, dtype=torch.int64, device="cuda")
        if noalloc:
            ctx.decode_noalloc(data, sbo_d, nseg, max_ids, out, off)
        else:
            ctx.decode(data, sbo_d, nseg, max_ids, out, off)
        st = ctx.sync_status()
        off_h = off.cpu().numpy().view(np.uint64)
        n = int(off_h[-1]) if st == 0 else 0
        res.append((st, out[:n].cpu().numpy().view(np.uint32).copy(), off_h.copy()))
    return res


def level_batch(scale, nseg, seed):
    """The largest BFS level of an R-MAT graph, split into Zipf ranges (many
    empty and short segments: raw and empty forms included)."""
    g = inputs.graph(inputs.RMAT, scale, 16, seed)
    level, _, depth = oracle.bfs(g, int(inputs.roots(g, 1, seed)[0]))
    L = int(np.argmax([np.sum(level == x) for x in range(depth + 1)]))
    zb, _ = inputs.bounds_zipf(g.n_vertices, nseg, seed)
    return oracle.batch_from_frontier(oracle.frontier(level, L), zb, L)


def test_noalloc_decode_equals_workspace_decode_twice(ctx):
    # first call: many segments and IDs; second: fewer of both, so the
    # scratch array still holds the first call's larger plan
    cases = [("rmat-s16-zipf1024", level_batch(16, 1024, 1)),
             ("rmat-s14-zipf40", level_batch(14, 40, 2))]
    assert cases[1][1].nseg < cases[0][1].nseg and cases[1][1].n_ids < cases[0][1].n_ids
    for name, b in cases:
        log("noalloc decode: %s, %d IDs in %d segments" % (name, b.n_ids, b.nseg))
        st, stream, sbo = gpu_encode(ctx, b)
        assert st == 0
        (st_w, ids_w, off_w), (st_n, ids_n, off_n) = both_decodes(ctx, stream, sbo, b.n_ids)
        assert st_w == 0 and st_n == 0
        assert np.array_equal(off_n, off_w), name
        assert np.array_equal(ids_n, ids_w), name
        want_st, want, want_off = oracle.decode(stream, sbo)
        assert want_st == 0
        assert np.array_equal(ids_n, want) and np.array_equal(off_n, want_off), name
        assert np.array_equal(ids_n, b.ids), name


def test_noalloc_decode_reports_what_decode_reports(ctx):
    """A stream with a flipped payload bit: both entry points latch the same
    status, and a too-small output capacity latches CAPACITY in both."""
    b = level_batch(12, 8, 3)
    st, stream, sbo = gpu_encode(ctx, b)
    assert st == 0
    # flip a bit in the last payload word of the largest compressed segment
    r = int(np.argmax(np.diff(sbo.astype(np.int64))))
    bad = stream.copy()
    bad[int(sbo[r + 1]) - 2] ^= 0x10
    (st_w, _, _), (st_n, _, _) = both_decodes(ctx, bad, sbo, b.n_ids)
    want_st, _, _ = oracle.decode(bad, sbo)
    assert st_w == st_n
    assert (st_w == 0) == (want_st == 0)
    (st_w, _, _), (st_n, _, _) = both_decodes(ctx, stream, sbo, b.n_ids - 1)
    assert st_w == st_n != 0


def test_noalloc_decode_refuses_too_many_segments(ctx):
    """More segments than the scratch array holds is refused on the host,
    before anything is enqueued."""
    import torch
    import paper_1704_00513_amd as P
    nseg = P.DECODE_NOALLOC_MAX_SEGS + 1
    data = torch.zeros(64, dtype=torch.uint8, device="cuda")
    sbo = torch.zeros(nseg + 1, dtype=torch.int64, device="cuda")
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    off = torch.zeros(nseg + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(P.BfscError) as e:
        ctx.decode_noalloc(data, sbo, nseg, 16, out, off)
    assert e.value.status == P.E_INVAL
    # the largest allowed count works: all segments empty
    nseg = P.DECODE_NOALLOC_MAX_SEGS
    ctx.decode_noalloc(data, sbo[:nseg + 1], nseg, 16, out, off[:nseg + 1])
    assert ctx.sync_status() == 0
    assert int(off[:nseg + 1].abs().sum().item()) == 0
