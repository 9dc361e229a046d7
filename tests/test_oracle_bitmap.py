"""Pins of the oracle's bitmap codec (one owner's share of a vertex bitmap,
coded block by block: ZERO, ONES, SET list, CLEAR list, LITERAL).

Nothing here calls the oracle to check the oracle: an independent reader
and writer of the format, written below from the format description with
Python integers as bit strings, checks the oracle's streams and its choice;
worked examples give hand-computed bytes; special cases reduce to a closed
form."""
import numpy as np
import pytest

import oracle

BW = 128  # words per block


def words_of(bits):
    """bool[32 n] -> u32[n], bit i is bit (i mod 32) of word i / 32."""
    b = np.asarray(bits, bool).reshape(-1, 32)
    return (b.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)


def bits_of(words):
    w = np.asarray(words, np.uint32).astype(np.uint64)
    return ((w[:, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(bool).reshape(-1)


def py_block_sizes(block_words):
    """Payload words of SET, CLEAR and LITERAL for one block, from the
    positions found with numpy (independent of the oracle)."""
    b = bits_of(block_words)
    out = {}
    for name, want in (("set", True), ("clear", False)):
        pos = np.nonzero(b == want)[0]
        if pos.size == 0:
            out[name] = None
            continue
        gmax = int(np.diff(pos).max()) if pos.size > 1 else 0
        width = gmax.bit_length()
        out[name] = ((pos.size - 1) * width + 31) // 32
    out["literal"] = len(block_words)
    return out


def py_read(stream, sbo):
    """Independent reader: a segment's bytes as one Python integer; fields
    taken by shifting.  Returns the decoded words of all segments."""
    data = bytes(stream)
    res = []
    for r in range(len(sbo) - 1):
        s, e = int(sbo[r]), int(sbo[r + 1])
        if s == e:
            continue
        seg = data[s:e]
        u32 = lambda o: int.from_bytes(seg[o:o + 4], "little")
        nw, pop, nb, magic = u32(0), u32(4), u32(8), u32(12)
        assert magic == 0x31434D42 and nb == (nw + BW - 1) // BW
        meta = 16 + 12 * nb
        pay = int.from_bytes(seg[meta:], "little")
        total_pay = (len(seg) - meta) // 4
        words = []
        prev_end = 0
        for k in range(nb):
            d = seg[16 + 12 * k:16 + 12 * k + 12]
            off = int.from_bytes(d[0:4], "little")
            count = int.from_bytes(d[4:6], "little")
            first = int.from_bytes(d[6:8], "little")
            cls, width = d[8], d[9]
            assert d[10:12] == b"\0\0" and off == prev_end
            n32 = min(BW, nw - BW * k)
            bp = pay >> (32 * off)
            if cls == 0:
                blk, used = [0] * n32, 0
            elif cls == 1:
                blk, used = [0xFFFFFFFF] * n32, 0
            elif cls == 4:
                blk, used = [(bp >> (32 * i)) & 0xFFFFFFFF for i in range(n32)], n32
            else:
                x = 0
                p = first
                x |= 1 << p
                for j in range(1, count):
                    p += (bp >> ((j - 1) * width)) & ((1 << width) - 1)
                    x |= 1 << p
                if cls == 3:
                    x = ((1 << (32 * n32)) - 1) ^ x
                blk = [(x >> (32 * i)) & 0xFFFFFFFF for i in range(n32)]
                used = ((count - 1) * width + 31) // 32
            words.extend(blk)
            prev_end = off + used
        assert prev_end == total_pay
        assert sum(bin(w).count("1") for w in words) == pop
        res.extend(words)
    return np.array(res, np.uint32)


def random_bitmap(n_words, density, seed, runs=False):
    rng = np.random.default_rng(seed)
    if not runs:
        return words_of(rng.random(32 * n_words) < density)
    # runs of ones and zeros, as in a visited bitmap of clustered IDs
    b = np.zeros(32 * n_words, bool)
    i, on = 0, bool(rng.integers(0, 2))
    while i < b.size:
        ln = int(rng.geometric(1.0 / 900))
        b[i:i + ln] = on if rng.random() > 0.1 else rng.random(min(ln, b.size - i)) < density
        i += ln
        on = not on
    return words_of(b)


@pytest.mark.parametrize("density", [0.0, 0.002, 0.05, 0.3, 0.5, 0.8, 0.97, 0.999, 1.0])
def test_round_trip_and_independent_reader(density):
    w = random_bitmap(700, density, int(density * 1000) + 1)
    seg_w = np.array([0, 1, 129, 129, 400, 700], np.uint64)  # one-word, exact block, empty, ragged
    stream, sbo = oracle.bmc_encode(w, seg_w)
    st, back, off = oracle.bmc_decode(stream, sbo)
    assert st == 0 and np.array_equal(back, w) and np.array_equal(off, seg_w)
    assert np.array_equal(py_read(stream, sbo), w)


def test_clustered_runs_use_every_class():
    w = random_bitmap(4000, 0.3, 7, runs=True)
    seg_w = np.array([0, 1000, 2500, 4000], np.uint64)
    stream, sbo = oracle.bmc_encode(w, seg_w)
    assert np.array_equal(py_read(stream, sbo), w)
    cls = oracle.bmc_classes(w, seg_w)
    assert set(cls.tolist()) >= {0, 1, 2, 3, 4}


def test_choice_is_the_smallest_under_the_tie_order():
    """Brute force: the sizes of SET, CLEAR and LITERAL measured from the
    positions (numpy) for every block; ZERO / ONES exactly when a list is
    empty; else the minimum with ties SET < CLEAR < LITERAL."""
    rng = np.random.default_rng(3)
    for trial in range(300):
        n32 = int(rng.integers(1, BW + 1))
        dens = float(rng.choice([0.001, 0.01, 0.1, 0.5, 0.9, 0.99, 0.999]))
        w = random_bitmap(n32, dens, 1000 + trial, runs=bool(trial % 2))
        seg_w = np.array([0, n32], np.uint64)
        got = int(oracle.bmc_classes(w, seg_w)[0])
        sz = py_block_sizes(w)
        if sz["set"] is None:
            want = 0
        elif sz["clear"] is None:
            want = 1
        else:
            order = [(sz["set"], 0, 2), (sz["clear"], 1, 3), (sz["literal"], 2, 4)]
            want = min(order)[2]
        assert got == want, (trial, sz, got)
        stream, sbo = oracle.bmc_encode(w, seg_w)
        cost = {0: 0, 1: 0, 2: sz["set"], 3: sz["clear"], 4: sz["literal"]}[got]
        assert int(sbo[-1]) == 16 + 12 + 4 * cost


def test_worked_examples():
    # one word, bits 0, 5 and 7: SET, count 3, first 0, gaps 5 and 2 at
    # width bitlen(5) = 3 -> payload 5 | 2 << 3 = 21 in one word
    w = np.array([(1 << 0) | (1 << 5) | (1 << 7)], np.uint32)
    stream, sbo = oracle.bmc_encode(w, np.array([0, 1], np.uint64))
    want = (
        (1).to_bytes(4, "little") + (3).to_bytes(4, "little") + (1).to_bytes(4, "little")
        + (0x31434D42).to_bytes(4, "little")
        + (0).to_bytes(4, "little") + (3).to_bytes(2, "little") + (0).to_bytes(2, "little")
        + bytes([2, 3]) + b"\0\0"
        + (21).to_bytes(4, "little"))
    assert bytes(stream) == want
    # all ones but bit 9 of the second word: CLEAR with one position, no payload
    w = np.array([0xFFFFFFFF, 0xFFFFFFFF ^ (1 << 9)], np.uint32)
    stream, sbo = oracle.bmc_encode(w, np.array([0, 2], np.uint64))
    d = bytes(stream[16:28])
    assert int(sbo[-1]) == 28 and d[8] == 3 and int.from_bytes(d[4:6], "little") == 1
    assert int.from_bytes(d[6:8], "little") == 41 and d[9] == 0
    # zero and full blocks take their 12-byte directory entry only
    w = np.concatenate([np.zeros(BW, np.uint32), np.full(BW, 0xFFFFFFFF, np.uint32)])
    stream, sbo = oracle.bmc_encode(w, np.array([0, 2 * BW], np.uint64))
    assert int(sbo[-1]) == 16 + 24
    assert list(oracle.bmc_classes(w, np.array([0, 2 * BW], np.uint64))) == [0, 1]


def test_literal_when_lists_do_not_pay():
    # alternating bits: every gap 2 (width 2) for 2048 positions -> 64 words
    # each list, 128 literal words ... lists win; a random half-dense block
    # has gaps up to ~20 -> lists of ~2048 x 5 bits = 320 words > 128
    w = np.full(BW, 0x55555555, np.uint32)
    assert int(oracle.bmc_classes(w, np.array([0, BW], np.uint64))[0]) == 2
    w = random_bitmap(BW, 0.5, 11)
    assert int(oracle.bmc_classes(w, np.array([0, BW], np.uint64))[0]) == 4


def test_damaged_streams_are_rejected_or_exact():
    """Single-bit flips: the oracle either rejects the stream or decodes
    exactly what the independent reader decodes from the same bytes."""
    w = random_bitmap(600, 0.3, 5, runs=True)
    seg_w = np.array([0, 300, 600], np.uint64)
    stream, sbo = oracle.bmc_encode(w, seg_w)
    rng = np.random.default_rng(8)
    rejected = 0
    for trial in range(300):
        s = stream.copy()
        pos = int(rng.integers(0, s.size))
        s[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        st, back, _ = oracle.bmc_decode(s, sbo)
        if st != 0:
            rejected += 1
            continue
        try:
            ref = py_read(s, sbo)
        except (AssertionError, IndexError):
            pytest.fail("oracle accepted a stream the reader rejects (trial %d)" % trial)
        assert np.array_equal(back, ref)
    assert rejected > 100


def test_bound_holds():
    for dens in (0.0, 0.5, 1.0):
        w = random_bitmap(1000, dens, 2)
        seg_w = np.array([0, 1, 130, 1000], np.uint64)
        stream, sbo = oracle.bmc_encode(w, seg_w)
        assert int(sbo[-1]) <= oracle.bmc_bound(1000, 3)
