"""GPU parity of the context settings (bfsc_config) and of the segment forms
they select, through the C-ABI:

- the compression threshold ("Usage of compression thresholds" section):
  streams byte-equal to the oracle's for thresholds 0, 1, the default, 200
  and the largest, in both plain and exhaustive choice and the fused learned
  pass; mixed batches of empty, raw and compressed segments; raw segments
  with unsorted or out-of-range IDs refused like the oracle; damaged raw
  segments accepted or refused as the oracle does;
- literal resolve of the learned widths against oracle.resolve(literal=True);
- bfsc_mlp_init against the seeded generator's weights;
- BFSC_SEL_DEFAULT and the launch-shape cache file.
"""
import os

import numpy as np
import pytest

import inputs
import oracle
from oracle import Batch
from oracle import mlp

from gpu_util import gpu_decode, gpu_encode, gpu_select, torch
from test_gpu_codec import batches

pytestmark = pytest.mark.gpu

THRESHOLDS = [0, 1, oracle.RAW_BELOW, 200, 2048]


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def contexts():
    import paper_1704_00513_amd as P
    cs = {T: P.Context(0, raw_below=T) for T in THRESHOLDS}
    yield cs
    for c in cs.values():
        c.close()


def mixed_batch(seed=8):
    rng = np.random.default_rng(seed)
    sizes = [0, 1, 31, 32, 0, 500, 7, 0, 129, 199, 200, 2047, 2048, 3000, 2, 0]
    segs, lo, hi = [], [], []
    base = 0
    for n in sizes:
        segs.append(np.sort(rng.choice(1 << 16, n, replace=False)).astype(np.uint32) + base)
        lo.append(base)
        hi.append(base + (1 << 16))
        base += 1 << 16
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    return Batch(np.concatenate(segs), off, lo, hi, np.arange(len(sizes)) % 9)


def all_batches():
    return batches() + [("mixed", mixed_batch())]


@pytest.mark.parametrize("T", THRESHOLDS)
def test_threshold_streams_are_byte_exact(contexts, T):
    ctx = contexts[T]
    assert ctx.config()["raw_below"] == T
    for name, b in all_batches():
        for mode in (oracle.PLAIN_BP, oracle.EXHAUSTIVE):
            log("threshold T=%d mode=%d case=%s" % (T, mode, name))
            want, want_off = oracle.encode(b, mode=mode, raw_below=T)
            st, got, got_off = gpu_encode(ctx, b, mode=mode)
            assert st == 0, name
            np.testing.assert_array_equal(got_off, want_off, err_msg=name)
            np.testing.assert_array_equal(got, want, err_msg=name)
        st, ids, off = gpu_decode(ctx, want, want_off)
        assert st == 0, name
        np.testing.assert_array_equal(ids, b.ids, err_msg=name)
        np.testing.assert_array_equal(off, b.seg_off, err_msg=name)


@pytest.mark.parametrize("T", [0, oracle.RAW_BELOW, 2048])
def test_threshold_with_fused_learned_pass(contexts, T):
    # the fused learned pass skips raw segments too; its stream is the
    # oracle's encoding of the classes in its own directory entries
    ctx = contexts[T]
    ctx.mlp_set_weights(inputs.mlp_init(3))
    for name, b in all_batches():
        log("threshold learned T=%d case=%s" % (T, name))
        st, got, got_off = gpu_encode(ctx, b, mode=2)
        assert st == 0, name
        st2, cls, _ = gpu_select(ctx, b, 2)
        assert st2 == 0
        want, want_off = oracle.encode(b, classes=cls, raw_below=T)
        np.testing.assert_array_equal(got_off, want_off, err_msg=name)
        np.testing.assert_array_equal(got, want, err_msg=name)


@pytest.mark.parametrize("T", [oracle.RAW_BELOW, 2048])
def test_raw_segments_are_checked(contexts, T):
    ctx = contexts[T]
    log("raw input checks T=%d" % T)
    assert gpu_encode(ctx, Batch(np.array([5, 5, 9], np.uint32), [0, 3], [0], [100], [0]))[0] == 1
    assert gpu_encode(ctx, Batch(np.array([9, 5], np.uint32), [0, 2], [0], [100], [0]))[0] == 1
    assert gpu_encode(ctx, Batch(np.array([1, 2, 300], np.uint32), [0, 3], [0], [100], [0]))[0] == 1
    assert gpu_encode(ctx, Batch(np.array([4, 7], np.uint32), [0, 2], [5], [100], [0]))[0] == 1
    # a long raw segment (over 64 IDs: the check carries across the wave's
    # chunks) with one repeat in its second chunk
    ids = np.arange(0, 600, 3).astype(np.uint32)
    ids[100] = ids[99]
    if T > ids.size:
        assert gpu_encode(ctx, Batch(ids, [0, ids.size], [0], [1000], [0]))[0] == 1
    # still usable afterwards
    st, got, _ = gpu_encode(ctx, Batch(np.array([1, 2, 3], np.uint32), [0, 3], [0], [100], [0]))
    assert st == 0 and np.array_equal(got.view(np.uint32), [1, 2, 3])


def test_damaged_raw_segments_agree_with_oracle(contexts):
    ctx = contexts[2048]
    rng = np.random.default_rng(4)
    b = mixed_batch(9)
    stream, sbo = oracle.encode(b, raw_below=2048)
    for trial in range(80):
        s = stream.copy()
        pos = int(rng.integers(0, s.size))
        s[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        want_st, want_ids, want_off = oracle.decode(s, sbo)
        log("damaged raw trial=%d pos=%d oracle=%d" % (trial, pos, want_st))
        st, ids, off = gpu_decode(ctx, s, sbo)
        assert (st == 0) == (want_st == 0), (trial, st, want_st)
        if st == 0:
            np.testing.assert_array_equal(ids, want_ids)
            np.testing.assert_array_equal(off, want_off)
    # a segment length that is not a whole number of words, and equal words
    # 1 and 2: neither form
    bad_off = sbo.copy()
    bad_off[2] += np.uint64(2)
    assert gpu_decode(ctx, stream, bad_off)[0] == 3


def test_literal_resolve_matches_oracle():
    import paper_1704_00513_amd as P
    ctx = P.Context(0, resolve_literal=True)
    assert ctx.config()["resolve_literal"]
    theta = inputs.mlp_init(11)
    ctx.mlp_set_weights(theta)
    try:
        for name, b in batches()[:4] + [("mixed", mixed_batch())]:
            log("literal resolve case=%s" % name)
            st, got, fb = gpu_select(ctx, b, 2)
            assert st == 0
            F = oracle.features(b)
            z, _ = mlp.forward(theta.astype(np.float64), mlp.features_to_f64(F))
            pred = mlp.predict(theta.astype(np.float64), mlp.features_to_f64(F))
            want, want_fb = oracle.resolve(b, pred, literal=True)
            top2 = np.sort(z, axis=1)[:, -2:]
            clear = (top2[:, 1] - top2[:, 0]) > 2e-3 * (1 + np.abs(top2[:, 1]))
            np.testing.assert_array_equal(got[clear], want[clear], err_msg=name)
            if clear.all():
                assert fb == want_fb
            # the learned encode runs the literal selection first: its
            # stream is the oracle's encoding of those classes
            st, stream, sbo = gpu_encode(ctx, b, mode=2)
            assert st == 0
            ref, ref_off = oracle.encode(b, classes=got)
            np.testing.assert_array_equal(sbo, ref_off)
            np.testing.assert_array_equal(stream, ref)
    finally:
        ctx.close()


def test_mlp_init_equals_the_seeded_generator():
    import paper_1704_00513_amd as P
    ctx = P.Context(0)
    try:
        for seed in (1, 4, 12345):
            ctx.mlp_init(seed)
            np.testing.assert_array_equal(ctx.mlp_get_weights(), inputs.mlp_init(seed))
    finally:
        ctx.close()


def test_default_selector_and_tune_cache(tmp_path):
    import paper_1704_00513_amd as P
    t = torch()
    name, b = batches()[2]
    ctx = P.Context(0, selector=P.SEL_PLAIN_BP)
    try:
        st, got, off = gpu_encode(ctx, b, mode=P.SEL_DEFAULT)
        assert st == 0
        want, want_off = oracle.encode(b, mode=oracle.PLAIN_BP)
        np.testing.assert_array_equal(got, want)
    finally:
        ctx.close()
    path = str(tmp_path / "tune.txt")
    ctx = P.Context(0, autotune=True, tune_cache=path)
    try:
        from gpu_util import device_batch
        db = device_batch(b)
        ctx.autotune(db)
        tuned = ctx.get_tune()
    finally:
        ctx.close()
    line = open(path).read().split()
    assert len(line) == 8 and int(line[1]) > 0
    assert [int(x) for x in line[2:]] == [tuned[k] for k in ("enc_waves", "enc_wg_per_cu", "dec_waves",
                                                             "dec_wg_per_cu", "enc_pack", "dec_mode")]
    ctx = P.Context(0, autotune=True, tune_cache=path)
    try:
        assert ctx.get_tune() == tuned
        assert ctx.config()["tune_cache"] == path
    finally:
        ctx.close()
    # without autotune the file is not read
    plain = P.Context(0)
    ctx = P.Context(0, tune_cache=path)
    try:
        assert ctx.get_tune() == plain.get_tune()
    finally:
        ctx.close()
        plain.close()
