"""Whole-tile and whole-group units.  The pack passes give a wave whole tiles
(16 blocks), and the decoder whole groups, when the batch holds at least eight
per wave; small batches take half units.  The tests force the large-batch
forms on a batch of a few million IDs by shrinking the pack grid (one
workgroup of one wave per CU: 256 waves, so 2,048 tiles suffice) and by
handing the decoder a capacity that selects whole groups, and check the
streams byte for byte against the oracle (plain and exhaustive choice) and
against the two-pass learned encoding, the IDs after decoding, and damaged
streams against the oracle's reader."""
import numpy as np
import pytest

import inputs
import oracle
from oracle import Batch

from gpu_util import gpu_decode, gpu_encode, gpu_select

pytestmark = pytest.mark.gpu

GROUP_MAX_IDS = 1 << 28  # a capacity of 131,072 groups: whole-group decode units


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


def big_batch():
    """About 4.7 M IDs over [0, 2^28): dense runs (bitmaps), a sparse random
    range (bit-pack and PFOR), a raw segment, an empty one, ragged tails."""
    parts = []
    bounds = [0, 1 << 25, (1 << 25) + 40, 1 << 26, (1 << 26) + 100, 3 << 26, 1 << 28]
    parts.append(inputs.clustered_sorted(2_100_000, 1 << 25, 31, lo=0, runs=64))
    parts.append(inputs.random_sorted(17, 40, 32, lo=bounds[1]))                      # raw
    parts.append(inputs.random_sorted(1_300_001, bounds[3] - bounds[2], 33, lo=bounds[2]))
    parts.append(np.zeros(0, np.uint32))                                             # empty
    parts.append(inputs.clustered_sorted(900_123, bounds[5] - bounds[4], 34, lo=bounds[4], runs=9))
    parts.append(inputs.random_sorted(400_000, bounds[6] - bounds[5], 35, lo=bounds[5]))
    ids = np.concatenate(parts).astype(np.uint32)
    off = np.concatenate([[0], np.cumsum([p.size for p in parts])])
    nseg = len(parts)
    return Batch(ids, off, bounds[:-1], bounds[1:], [3] * nseg)


@pytest.fixture(scope="module")
def batch():
    b = big_batch()
    print("units batch: %d IDs in %d segments" % (b.n_ids, b.nseg), flush=True)
    return b


def _small_grid(ctx, **kw):
    before = ctx.get_tune()
    ctx.set_tune(enc_waves=1, enc_wg_per_cu=1, **kw)
    return before


@pytest.mark.parametrize("mode", [0, 1])
def test_whole_tile_pack_and_whole_group_decode(ctx, batch, mode):
    print("whole tiles mode=%d" % mode, flush=True)
    before = _small_grid(ctx)
    try:
        st, got, sbo = gpu_encode(ctx, batch, mode=mode)
    finally:
        ctx.set_tune(**before)
    assert st == 0
    want, want_sbo = oracle.encode(batch, mode=mode)
    np.testing.assert_array_equal(sbo, want_sbo)
    np.testing.assert_array_equal(got, want)
    for max_ids in (None, GROUP_MAX_IDS):
        print("decode max_ids=%s" % max_ids, flush=True)
        st, ids, off = gpu_decode(ctx, got, sbo, max_ids=max_ids or batch.n_ids, out_cap=batch.n_ids)
        assert st == 0
        np.testing.assert_array_equal(ids, batch.ids)
        np.testing.assert_array_equal(off, np.asarray(batch.seg_off, np.uint64))


def test_whole_tile_fused_learned_equals_two_pass(ctx, batch):
    import os
    from test_selector_trained import WEIGHTS
    if not os.path.exists(WEIGHTS):
        pytest.skip("selector not trained")
    ctx.mlp_set_weights(np.load(WEIGHTS, allow_pickle=False))
    st, cls, _ = gpu_select(ctx, batch, 2)
    assert st == 0
    st, two, two_off = gpu_encode(ctx, batch, classes=cls)
    assert st == 0
    before = _small_grid(ctx)
    try:
        print("whole tiles fused learned", flush=True)
        st, fused, fused_off = gpu_encode(ctx, batch, mode=2)
    finally:
        ctx.set_tune(**before)
    assert st == 0
    np.testing.assert_array_equal(fused_off, two_off)
    np.testing.assert_array_equal(fused, two)
    want, _ = oracle.encode(batch, classes=cls)
    np.testing.assert_array_equal(fused, want)
    st, ids, _ = gpu_decode(ctx, fused, fused_off, max_ids=GROUP_MAX_IDS, out_cap=batch.n_ids)
    assert st == 0
    np.testing.assert_array_equal(ids, batch.ids)


def test_whole_group_decode_of_damaged_streams_agrees_with_oracle(ctx):
    """Whole-group units on damaged streams: accepted exactly when the
    oracle's reader accepts, with the same IDs."""
    rng = np.random.default_rng(41)
    ids = inputs.clustered_sorted(70_000, 1 << 22, 42, runs=6)
    gaps = np.full(40_000, 5, np.int64)
    gaps[::61] = 1 << 12
    pf = (1 << 23) + np.concatenate([[0], np.cumsum(gaps)])
    ids = np.concatenate([ids, pf]).astype(np.uint32)
    b = oracle.batch_from_frontier(ids, np.array([0, 1 << 22, 1 << 24], np.uint32), 2)
    stream, sbo = oracle.encode(b)
    for trial in range(40):
        s = stream.copy()
        for _ in range(int(rng.integers(1, 4))):
            pos = int(rng.integers(0, s.size))
            s[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        want_st, want_ids, want_off = oracle.decode(s, sbo)
        st, got, off = gpu_decode(ctx, s, sbo, max_ids=GROUP_MAX_IDS, out_cap=16 * s.size + 1)
        assert (st == 0) == (want_st == 0), (trial, st, want_st)
        if st == 0:
            np.testing.assert_array_equal(got, want_ids)
            np.testing.assert_array_equal(off, want_off)
