"""Pins of the oracle codec against what the paper and the mathematics fix:
worked examples (eqs. 6-9), round-trip identity (lossless requirement),
brute-force optimality over actually encoded candidates, an independent
bit-string reader of the format, and rejection of damaged streams."""
import struct

import numpy as np
import pytest

import inputs
import oracle
from oracle import Batch

BLOCK = 128


def one_segment(ids, lo=0, hi=None, level=0):
    ids = np.asarray(ids, np.uint32)
    if hi is None:
        hi = int(ids.max()) + 1 if ids.size else lo + 1
    return Batch(ids, [0, ids.size], [lo], [hi], [level])


def roundtrip(b, classes=None, mode=oracle.EXHAUSTIVE, raw_below=oracle.RAW_BELOW):
    stream, sbo = oracle.encode(b, classes, mode, raw_below=raw_below)
    st, out, off = oracle.decode(stream, sbo)
    assert st == oracle.ST_OK
    np.testing.assert_array_equal(out, b.ids)
    np.testing.assert_array_equal(off, b.seg_off)
    return stream, sbo


# ------------------------------------------------------------ worked examples

def test_eq7_width_of_2000_to_2127():
    # eq. (7): 128 integers in [2000, 2127] need ceil(log2(2127 + 1 - 2000)) = 7 bits
    assert oracle.bitlen(2127 - 2000) == 7


def test_eq9_width_rounds_up():
    # eq. (9): log2(990 + 1 - 5) = 9.95, printed "9,9"; a width is whole bits -> 10
    assert np.log2(990 + 1 - 5) == pytest.approx(9.945, abs=1e-3)
    assert oracle.bitlen(990 - 5) == 10


def test_eq7_block_as_deltas_ties_bitpack_and_bitmap():
    # The block 2000..2127 delta-coded: 127 gaps of 1 -> width 1, 127 bits = 4 words;
    # as a bitmap the span 127 also needs 4 words; the tie goes to bit-packing.
    b = one_segment(np.arange(2000, 2128), lo=0, hi=4096)
    cls = oracle.select(b)
    assert list(cls) == [2]  # BP width 1
    d = oracle.block_details(b, [0])
    assert d["words"][0] == 4 and d["span"][0] == 127
    d = oracle.block_details(b, [2])
    assert d["words"][0] == 4
    stream, sbo = roundtrip(b)
    # header 16 + directory 8 + group table 4 + 4 payload words
    assert int(sbo[-1]) == 16 + 8 + 4 + 16


def test_eq8_analog_outlier_becomes_exception():
    # eq. (8): one huge value among small ones ruins a plain frame of reference.
    # Sorted uint32 analog: 127 gaps of 3 then one gap of 2^30.
    ids = np.concatenate([np.arange(128 - 1) * 3, [126 * 3 + (1 << 30)]]).astype(np.uint32)
    b = one_segment(ids)
    assert list(oracle.select(b)) == [oracle.CLS_PFOR]
    d = oracle.block_details(b)
    # width 31 plain: ceil(127*31/32) = 124 words; PFOR b=2: 8 low + 1 pos + 1 high = 10 words
    assert d["wmin"][0] == 31
    assert d["pfor_b"][0] == 2 and d["pfor_e"][0] == 1
    assert d["words"][0] == 10
    stream, sbo = roundtrip(b)
    entry = stream[16:24]
    first, cls, param, aux = struct.unpack("<IBBH", entry.tobytes())
    assert (cls, param, aux & 0xFF, aux >> 8) == (34, 2, 1, 29)


def test_single_id_block_is_width_zero():
    b = one_segment([12345], lo=0, hi=20000)
    assert list(oracle.select(b)) == [1]
    stream, sbo = roundtrip(b, raw_below=0)
    assert int(sbo[-1]) == 16 + 8 + 4  # no payload words
    assert struct.unpack("<IIII", stream[:16].tobytes()) == (1, 20000, 0, 0x31434642)


def test_empty_segment_is_no_bytes():
    # whatever the threshold, an empty segment takes no bytes
    for T in (0, 1, oracle.RAW_BELOW):
        b = Batch(np.zeros(0, np.uint32), [0, 0], [0], [10])
        stream, sbo = roundtrip(b, raw_below=T)
        assert int(sbo[-1]) == 0 and stream.size == 0


# ------------------------------------------------------------ independent reader

def bits_of(words):
    """Stream bit i = bit (i mod 32) of word i/32, as a Python string."""
    return "".join(format(int(w), "032b")[::-1] for w in words)


def read_field(bits, pos, width):
    return int(bits[pos:pos + width][::-1], 2) if width else 0


def string_decode(stream):
    """A second, bit-string based reading of one segment (no shared code with
    the C reader): returns the values."""
    words = np.frombuffer(stream.tobytes(), np.uint32)
    if words.size == 0:
        return np.zeros(0, np.uint64)
    if words.size < 4 or words[1] < words[2]:
        # raw: the IDs themselves
        assert (np.diff(words.astype(np.int64)) > 0).all()
        return words.astype(np.uint64)
    n, hi, lo, magic = (int(x) for x in words[:4])
    assert magic == 0x31434642
    nb = (n + BLOCK - 1) // BLOCK
    ng = (nb + 15) // 16
    payload = words[4 + 2 * nb + ng:]
    gtab = words[4 + 2 * nb:4 + 2 * nb + ng]
    out = []
    pw = 0
    for k in range(nb):
        if k % 16 == 0:
            assert int(gtab[k // 16]) == pw
        first = int(words[4 + 2 * k])
        e = int(words[4 + 2 * k + 1])
        cls, param, aux = e & 0xFF, (e >> 8) & 0xFF, e >> 16
        nk = min(BLOCK, n - BLOCK * k)
        m = nk - 1
        vals = [lo + first]
        if cls == 0:
            nwords = (aux + 31) // 32
            bits = bits_of(payload[pw:pw + nwords])
            vals += [lo + first + i + 1 for i in range(aux) if bits[i] == "1"]
        elif cls <= 33:
            w = cls - 1
            nwords = (m * w + 31) // 32
            bits = bits_of(payload[pw:pw + nwords])
            for j in range(m):
                vals.append(vals[-1] + read_field(bits, j * w, w))
        else:
            bb, E, h = param, aux & 0xFF, aux >> 8
            lw, qw, hw = (m * bb + 31) // 32, (E + 3) // 4, (E * h + 31) // 32
            nwords = lw + qw + hw
            low = bits_of(payload[pw:pw + lw])
            pos = bits_of(payload[pw + lw:pw + lw + qw])
            high = bits_of(payload[pw + lw + qw:pw + nwords])
            d = [read_field(low, j * bb, bb) for j in range(m)]
            for x in range(E):
                p = read_field(pos, 8 * x, 8)
                d[p] += read_field(high, x * h, h) << bb
            for j in range(m):
                vals.append(vals[-1] + d[j])
        out += vals
        pw += nwords
    assert pw == len(payload)
    return np.array(out, np.uint64)


@pytest.mark.parametrize("seed", range(6))
def test_independent_bitstring_reader_agrees(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 700))
    if seed % 2:
        ids = inputs.clustered_sorted(n, 1 << 20, seed)
    else:
        ids = inputs.random_sorted(n, int(rng.integers(n, 1 << 24)), seed)
    b = one_segment(ids, lo=0, hi=1 << 24)
    stream, _ = oracle.encode(b)
    np.testing.assert_array_equal(string_decode(stream), ids.astype(np.uint64))


def test_every_class_and_pfor_width_round_trips():
    # forced classes: each valid class on many blocks
    rng = np.random.default_rng(7)
    for trial in range(40):
        n = int(rng.integers(1, 129))
        span_max = int(rng.choice([n + 10, 5000, 1 << 20, 1 << 31]))
        ids = inputs.random_sorted(n, max(n, span_max), trial)
        if trial % 5 == 0 and n > 11:
            ids[-1] = np.uint32(0xFFFFFFFE)  # huge outlier at the top of the u32 range
            ids = np.unique(ids)
        b = one_segment(ids, lo=0, hi=0xFFFFFFFF)
        d = oracle.block_details(b)
        wmin = int(d["wmin"][0])
        for cls in [0] + list(range(1 + wmin, 34)) + [34]:
            if cls == 0 and d["span"][0] > 4096:
                continue
            stream, sbo = roundtrip(b, np.array([cls], np.uint8), raw_below=0)
            np.testing.assert_array_equal(string_decode(stream), ids.astype(np.uint64))


def test_top_of_u32_range():
    ids = np.array([0, 1, 0xFFFFFFF0, 0xFFFFFFFD], np.uint32)
    b = one_segment(ids, lo=0, hi=0xFFFFFFFE)
    for T in (0, oracle.RAW_BELOW):
        stream, _ = roundtrip(b, raw_below=T)
        np.testing.assert_array_equal(string_decode(stream), ids.astype(np.uint64))


# ------------------------------------------------------------ brute force

def subsets_of_16():
    segs = []
    for mask in range(1, 1 << 16):
        segs.append([i for i in range(16) if mask >> i & 1])
    return segs


def test_bruteforce_exhaustive_is_optimal_on_all_subsets_of_16():
    segs = subsets_of_16()
    ids = np.concatenate([np.array(s, np.uint32) for s in segs])
    off = np.zeros(len(segs) + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in segs])
    R = len(segs)
    b = Batch(ids, off, np.zeros(R, np.uint32), np.full(R, 16, np.uint32))
    # actual sizes of every candidate class, by encoding it
    sizes = np.full((R, 35), np.iinfo(np.int64).max, np.int64)
    maxgap = np.array([max(np.diff(s)) if len(s) > 1 else 0 for s in segs])
    wmin = np.array([int(x).bit_length() for x in maxgap])
    for cls in range(35):
        if 1 <= cls <= 33:
            valid = (cls - 1) >= wmin
        else:
            valid = np.ones(R, bool)
        sel = np.flatnonzero(valid)
        sub = Batch(np.concatenate([ids[off[i]:off[i + 1]] for i in sel]),
                    np.concatenate([[0], np.cumsum([off[i + 1] - off[i] for i in sel])]),
                    np.zeros(sel.size, np.uint32), np.full(sel.size, 16, np.uint32))
        stream, sbo = oracle.encode(sub, np.full(sel.size, cls, np.uint8), raw_below=0)
        st, out, _ = oracle.decode(stream, sbo)
        assert st == oracle.ST_OK
        np.testing.assert_array_equal(out, sub.ids)
        sizes[sel, cls] = np.diff(sbo.astype(np.int64))
    ex = oracle.select(b).astype(np.int64)
    best = sizes.min(axis=1)
    assert (sizes[np.arange(R), ex] == best).all()
    # tie rule: smallest-width bit-packing, then bitmap, then PFOR
    order = list(range(1, 34)) + [0, 34]
    want = np.array([next(c for c in order if sizes[i, c] == best[i]) for i in range(R)])
    np.testing.assert_array_equal(ex, want)
    # and the exhaustive stream is that size
    stream, sbo = oracle.encode(b, raw_below=0)
    np.testing.assert_array_equal(np.diff(sbo.astype(np.int64)), best)


def test_bruteforce_random_full_blocks():
    rng = np.random.default_rng(11)
    segs = []
    for t in range(300):
        kind = t % 3
        if kind == 0:
            s = inputs.random_sorted(128, int(rng.integers(128, 20000)), 1000 + t)
        elif kind == 1:
            s = inputs.clustered_sorted(128, 1 << 16, 1000 + t)
        else:
            gaps = rng.integers(1, 8, size=127)
            gaps[rng.integers(0, 127, size=int(rng.integers(1, 14)))] = rng.integers(1 << 10, 1 << 20)
            s = np.concatenate([[0], np.cumsum(gaps)]).astype(np.uint32)
        segs.append(s)
    for s in segs:
        b = one_segment(s, lo=0, hi=1 << 31)
        best, best_c = None, None
        order = list(range(1, 34)) + [0, 34]
        d = oracle.block_details(b)
        for c in order:
            if 1 <= c <= 33 and c - 1 < d["wmin"][0]:
                continue
            if c == 0 and d["span"][0] > 4096:
                continue
            stream, sbo = oracle.encode(b, np.array([c], np.uint8))
            sz = int(sbo[-1])
            if best is None or sz < best:
                best, best_c = sz, c
        assert int(oracle.select(b)[0]) == best_c


# ------------------------------------------------------------ size model

def test_size_model_matches_stream_and_bound():
    for seed in range(5):
        g = inputs.graph(inputs.RMAT, 12, 16, seed + 1)
        root = inputs.roots(g, 1, seed + 1)[0]
        level, parent, depth = oracle.bfs(g, root)
        bounds = inputs.bounds_equal(g.n_vertices, 4)
        for L in range(depth + 1):
            b = oracle.batch_from_frontier(oracle.frontier(level, L), bounds, L)
            for mode in (oracle.PLAIN_BP, oracle.EXHAUSTIVE):
                stream, sbo = roundtrip(b, mode=mode)
                assert oracle.encoded_size(b, mode=mode) == int(sbo[-1])
                assert int(sbo[-1]) <= oracle.encode_bound(b.n_ids, b.nseg)


def test_plain_is_never_smaller_than_exhaustive():
    ids = inputs.clustered_sorted(5000, 1 << 22, 3)
    b = oracle.batch_from_frontier(ids, inputs.bounds_equal(1 << 22, 7))
    assert oracle.encoded_size(b, mode=oracle.EXHAUSTIVE) <= oracle.encoded_size(b, mode=oracle.PLAIN_BP)


def test_capacity_and_invalid_inputs():
    b = one_segment(np.arange(0, 1000, 3))
    assert oracle.encode_status(b, cap=64)[0] == oracle.ST_CAPACITY
    bad = one_segment(np.array([5, 5, 7], np.uint32))  # not strictly increasing
    assert oracle.encode_status(bad)[0] == oracle.ST_INVAL
    out_of_range = Batch(np.array([1, 2, 30], np.uint32), [0, 3], [0], [20])
    assert oracle.encode_status(out_of_range)[0] == oracle.ST_INVAL
    # a forced class that cannot hold the block (in the compressed form)
    b = one_segment(np.array([0, 1000], np.uint32), hi=2000)
    assert oracle.encode_status(b, classes=np.array([3], np.uint8), raw_below=0)[0] == oracle.ST_INVAL


# ------------------------------------------------------------ damaged streams

def test_damaged_streams_are_rejected_not_misread():
    rng = np.random.default_rng(5)
    ids = inputs.clustered_sorted(3000, 1 << 20, 9)
    b = oracle.batch_from_frontier(ids, inputs.bounds_equal(1 << 20, 3))
    stream, sbo = oracle.encode(b)
    rejected = 0
    for t in range(400):
        s = stream.copy()
        pos = int(rng.integers(0, s.size))
        s[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        st, out, _ = oracle.decode(s, sbo)
        if st == oracle.ST_OK:
            # a flip inside a payload may still decode to a valid (different)
            # strictly increasing list; it must then differ from the input or
            # be a flip of padding that changes nothing
            assert out.size == ids.size
        else:
            assert st == oracle.ST_CORRUPT
            rejected += 1
    assert rejected > 100
    # truncation
    for cut in (1, 4, 17, stream.size // 2):
        sb = sbo.copy()
        sb[-1] -= np.uint64(cut)
        st, _, _ = oracle.decode(stream[:int(sb[-1])], sb)
        assert st == oracle.ST_CORRUPT
    # bad magic, bad class, bad width (single segment so offsets are known)
    stream, sbo = oracle.encode(one_segment(ids, lo=0, hi=1 << 20))
    s = stream.copy()
    s[12] ^= 0xFF
    assert oracle.decode(s, sbo)[0] == oracle.ST_CORRUPT
    s = stream.copy()
    s[16 + 4] = 200
    assert oracle.decode(s, sbo)[0] == oracle.ST_CORRUPT
    s = stream.copy()
    s[16 + 5] ^= 0x40  # param no longer matches the class
    assert oracle.decode(s, sbo)[0] == oracle.ST_CORRUPT


# ------------------------------------------------------------ entropy and ratio

def test_entropy_fair_coin_is_one_bit():
    # eq. (2) and its coin example: H = 1 for two equiprobable outcomes
    assert oracle.entropy(np.array([0, 1] * 500)) == pytest.approx(1.0)
    assert oracle.entropy(np.full(100, 7)) == 0.0
    assert oracle.entropy(np.arange(1024)) == pytest.approx(10.0)


def test_ratio_definitions():
    # eq. (4) ratio = original / compressed; eq. (10) ratio % = 100 / ratio
    assert oracle.ratio(400, 100) == 4.0
    assert oracle.ratio_percent(400, 100) == 25.0
