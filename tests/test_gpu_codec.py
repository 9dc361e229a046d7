"""GPU parity of the codec (select, encode, decode, features) against the CPU
oracle through the C-ABI: byte-exact streams, bit-exact IDs and classes."""
import numpy as np
import pytest

import inputs
import oracle
from oracle import Batch

from gpu_util import gpu_decode, gpu_encode, gpu_features, gpu_select, shifted_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


def log(msg):
    print(msg, flush=True)


def batches():
    """Seeded batches spanning several tiles, ragged tails and edge cases."""
    out = []
    # config-1 style: s16 R-MAT frontiers, one segment over [0, V)
    g = inputs.graph(inputs.RMAT, 16, 16, 1)
    root = int(inputs.roots(g, 1, 1)[0])
    level, parent, depth = oracle.bfs(g, root)
    for L in range(depth + 1):
        out.append(("s16-L%d" % L, oracle.batch_from_frontier(oracle.frontier(level, L),
                                                              np.array([0, g.n_vertices], np.uint32), L)))
    # 16 equal segments of an s16 uniform-graph level
    gu = inputs.graph(inputs.UNIFORM, 16, 16, 1)
    lu, _, du = oracle.bfs(gu, int(inputs.roots(gu, 1, 1)[0]))
    fr = [oracle.frontier(lu, L) for L in range(du + 1)]
    big = max(range(len(fr)), key=lambda i: fr[i].size)
    out.append(("uniform16-eq16", oracle.batch_from_frontier(fr[big], inputs.bounds_equal(gu.n_vertices, 16), big)))
    # Zipf segments, many empty or tiny
    zb, _ = inputs.bounds_zipf(g.n_vertices, 256, 1)
    f = oracle.frontier(level, int(np.argmax([np.sum(level == L) for L in range(depth + 1)])))
    out.append(("zipf256", oracle.batch_from_frontier(f, zb, 3)))
    # clustered and random sets with exceptions, crossing tile boundaries
    out.append(("clustered", oracle.batch_from_frontier(inputs.clustered_sorted(9000, 1 << 22, 5),
                                                        inputs.bounds_equal(1 << 22, 5), 1)))
    out.append(("random-sparse", oracle.batch_from_frontier(inputs.random_sorted(7000, 1 << 31, 6),
                                                            np.array([0, 1 << 31], np.uint32), 2)))
    # exact multiples of blocks / groups and one-past
    for n in (128, 2048, 2049, 4096 + 1, 1):
        out.append(("n%d" % n, oracle.batch_from_frontier(inputs.random_sorted(n, 1 << 20, n),
                                                          np.array([0, 1 << 20], np.uint32), 0)))
    # outliers that force PFOR, top of the u32 range
    gaps = np.full(4000, 3, np.int64)
    gaps[::137] = 1 << 27
    ids = np.concatenate([[5], 5 + np.cumsum(gaps)]).astype(np.uint32)
    out.append(("pfor", oracle.batch_from_frontier(ids, np.array([0, 0xFFFFFFFF], np.uint32), 4)))
    # PFOR with narrow exceptions (low and high parts within 24 bits) over
    # whole groups of full blocks
    gaps = np.full(6000, 5, np.int64)
    gaps[::97] = 1 << 19
    ids = np.concatenate([[7], 7 + np.cumsum(gaps)]).astype(np.uint32)
    out.append(("pfor24", oracle.batch_from_frontier(ids, np.array([0, 1 << 31], np.uint32), 4)))
    top = np.array([0, 1, 0xFFFFFF00, 0xFFFFFFF0, 0xFFFFFFFD], np.uint32)
    out.append(("top", Batch(top, [0, 5], [0], [0xFFFFFFFE], [0])))
    # all segments empty but one
    out.append(("mostly-empty", Batch(np.array([10, 20], np.uint32), [0, 0, 0, 0, 2], [0, 5, 8, 9],
                                      [5, 8, 9, 100], [0, 0, 0, 0])))
    return out


@pytest.mark.parametrize("pack", list(range(8)))
@pytest.mark.parametrize("waves", [2, 4, 16])
@pytest.mark.parametrize("mode", [oracle.PLAIN_BP, oracle.EXHAUSTIVE])
def test_encode_is_byte_exact(ctx, mode, waves, pack):
    before = ctx.get_tune()
    ctx.set_tune(enc_waves=waves, enc_pack=pack)
    try:
        for name, b in batches():
            log("encode mode=%d waves=%d pack=%d case=%s n=%d nseg=%d" % (mode, waves, pack, name,
                                                                         b.n_ids, b.nseg))
            want, want_off = oracle.encode(b, mode=mode)
            st, got, got_off = gpu_encode(ctx, b, mode=mode)
            assert st == 0, name
            np.testing.assert_array_equal(got_off, want_off, err_msg=name)
            np.testing.assert_array_equal(got, want, err_msg=name)
    finally:
        ctx.set_tune(**before)


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 6])
@pytest.mark.parametrize("waves", [2, 4, 8, 16])
def test_decode_shapes(ctx, waves, mode):
    before = ctx.get_tune()
    ctx.set_tune(dec_waves=waves, dec_mode=mode)
    try:
        for name, b in batches():
            log("decode waves=%d mode=%d case=%s" % (waves, mode, name))
            stream, sbo = oracle.encode(b)
            st, ids, off = gpu_decode(ctx, stream, sbo)
            assert st == 0
            np.testing.assert_array_equal(ids, b.ids)
    finally:
        ctx.set_tune(**before)


def test_select_matches_oracle(ctx):
    for name, b in batches():
        for mode in (oracle.PLAIN_BP, oracle.EXHAUSTIVE):
            log("select mode=%d case=%s" % (mode, name))
            st, got, _ = gpu_select(ctx, b, mode)
            assert st == 0
            np.testing.assert_array_equal(got, oracle.select(b, mode), err_msg=name)


def test_encode_with_given_classes(ctx):
    rng = np.random.default_rng(3)
    for name, b in batches()[:6] + batches()[-4:]:
        d = oracle.block_details(b)
        # a random valid class per block
        cls = []
        for wmin, span in zip(d["wmin"], d["span"]):
            opts = list(range(1 + int(wmin), 34)) + [34] + ([0] if span <= 4096 else [])
            cls.append(int(rng.choice(opts)))
        cls = np.array(cls, np.uint8)
        log("given-classes case=%s" % name)
        want, want_off = oracle.encode(b, classes=cls)
        st, got, got_off = gpu_encode(ctx, b, classes=cls)
        assert st == 0
        np.testing.assert_array_equal(got_off, want_off)
        np.testing.assert_array_equal(got, want)


def test_decode_is_exact(ctx):
    for name, b in batches():
        log("decode case=%s" % name)
        stream, sbo = oracle.encode(b)
        st, ids, off = gpu_decode(ctx, stream, sbo)
        assert st == 0, name
        np.testing.assert_array_equal(off, b.seg_off, err_msg=name)
        np.testing.assert_array_equal(ids, b.ids, err_msg=name)


def test_features_bit_exact(ctx):
    for name, b in batches():
        log("features case=%s" % name)
        st, got = gpu_features(ctx, b)
        assert st == 0
        np.testing.assert_array_equal(got, oracle.features(b), err_msg=name)


def test_invalid_input_is_reported(ctx):
    log("invalid-input")
    bad = Batch(np.array([5, 5, 9], np.uint32), [0, 3], [0], [100], [0])
    st, _, _ = gpu_encode(ctx, bad)
    assert st == 1
    out_of_range = Batch(np.array([1, 2, 300], np.uint32), [0, 3], [0], [100], [0])
    assert gpu_encode(ctx, out_of_range)[0] == 1
    b = batches()[2][1]  # a multi-block level: gaps of at least 1
    assert b.n_ids > 1000
    cls = np.full(b.n_blocks, 1, np.uint8)  # width 0 cannot hold real gaps
    assert gpu_encode(ctx, b, classes=cls)[0] == 1
    # still usable afterwards
    st, got, _ = gpu_encode(ctx, b)
    assert st == 0


@pytest.mark.parametrize("dec_mode", [3, 6])
def test_capacity_is_reported(ctx, dec_mode):
    name, b = batches()[3]
    log("capacity case=%s dec_mode=%d" % (name, dec_mode))
    st, _, _ = gpu_encode(ctx, b, out_cap=256)
    assert st == 2
    stream, sbo = oracle.encode(b)
    ctx.set_tune(dec_mode=dec_mode)
    try:
        st, _, _ = gpu_decode(ctx, stream, sbo, max_ids=b.n_ids, out_cap=b.n_ids // 2)
        assert st == 2
        # a stream holding more IDs than max_ids, with room in the output
        st, _, _ = gpu_decode(ctx, stream, sbo, max_ids=b.n_ids - 1, out_cap=b.n_ids)
        assert st == 2
        # and the exact bound is fine
        st, ids, _ = gpu_decode(ctx, stream, sbo, max_ids=b.n_ids, out_cap=b.n_ids)
        assert st == 0
        np.testing.assert_array_equal(ids, b.ids)
    finally:
        ctx.set_tune(dec_mode=3)


@pytest.mark.parametrize("dec_mode", [0, 1, 2, 3, 4, 6])
def test_damaged_streams_agree_with_oracle(ctx, dec_mode):
    ctx.set_tune(dec_mode=dec_mode)
    rng = np.random.default_rng(9)
    for name, b in [x for x in batches() if x[0] in ("clustered", "pfor", "pfor24", "s16-L3", "zipf256")]:
        stream, sbo = oracle.encode(b)
        log("damage case=%s bytes=%d" % (name, stream.size))
        for trial in range(60):
            s = stream.copy()
            for _ in range(int(rng.integers(1, 4))):
                pos = int(rng.integers(0, s.size))
                s[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
            want_st, want_ids, want_off = oracle.decode(s, sbo)
            st, ids, off = gpu_decode(ctx, s, sbo)
            assert (st == 0) == (want_st == 0), (name, trial, st, want_st)
            if st == 0:
                np.testing.assert_array_equal(ids, want_ids)
                np.testing.assert_array_equal(off, want_off)
    ctx.set_tune(dec_mode=3)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_unaligned_ids_and_output(ctx, shift):
    """IDs and decoded output at addresses that are not 16-byte aligned take
    the word-by-word paths of the row encoder and of the row decoder: the
    stream and the IDs are the same as from aligned buffers."""
    import paper_1704_00513_amd as P
    from gpu_util import torch
    t = torch()
    before = ctx.get_tune()
    try:
        for name, b in batches():
            if b.n_ids < 1024:
                continue
            db, keep = shifted_batch(b, shift)
            for mode in (oracle.PLAIN_BP, oracle.EXHAUSTIVE):
                log("unaligned encode shift=%d mode=%d case=%s" % (shift, mode, name))
                cap = P.Context.encode_bound(b.n_ids, b.nseg)
                out = t.zeros(cap, dtype=t.uint8, device="cuda")
                sbo = t.zeros(b.nseg + 1, dtype=t.int64, device="cuda")
                ctx.encode(db, out, sbo, mode=mode, out_cap=cap)
                assert ctx.sync_status() == 0
                sbo_h = sbo.cpu().numpy().view(np.uint64)
                want, want_off = oracle.encode(b, mode=mode)
                np.testing.assert_array_equal(sbo_h, want_off, err_msg=name)
                np.testing.assert_array_equal(out[:int(sbo_h[-1])].cpu().numpy(), want, err_msg=name)
            stream, sbo = oracle.encode(b)
            data = t.from_numpy(np.concatenate([stream, np.zeros(4, np.uint8)])).to("cuda")
            sbo_d = t.from_numpy(np.ascontiguousarray(sbo, np.uint64).view(np.int64)).to("cuda")
            for dec_mode in (3, 6):
                log("unaligned decode shift=%d dec_mode=%d case=%s" % (shift, dec_mode, name))
                ctx.set_tune(dec_mode=dec_mode)
                obuf = t.zeros(b.n_ids + shift + 4, dtype=t.int32, device="cuda")
                off = t.zeros(b.nseg + 1, dtype=t.int64, device="cuda")
                ctx.decode(data, sbo_d, b.nseg, b.n_ids, obuf[shift:shift + b.n_ids], off, out_cap=b.n_ids)
                assert ctx.sync_status() == 0
                got = obuf[shift:shift + b.n_ids].cpu().numpy().view(np.uint32)
                np.testing.assert_array_equal(got, b.ids, err_msg=name)
            del keep
    finally:
        ctx.set_tune(**before)
