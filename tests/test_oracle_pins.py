"""Pins of the oracle pieces that no worked example of the paper fixes:

- the PFOR exception width b (patched coding with exceptions, eqs. (8)-(9) of
  the compression-techniques section): fewest payload words among the b with
  at most one exception in ten deltas, ties to the larger b.  Checked by brute
  force over every b with a size function written here, on random blocks, on a
  block where two widths tie, and on one where a width with too many
  exceptions would be smaller;
- the PFOR block layout for every b, by streams assembled here field by field
  and read back by the oracle decoder;
- the fp16 rounding points of the selector network's forward pass (weights,
  and each hidden layer after bias and ReLU), by a network whose logits are
  worked out by hand and change if any one rounding is left out.
"""
import struct

import numpy as np
import pytest

import inputs
import oracle
from oracle import Batch
from oracle import mlp

M10 = 10  # at most one exception per ten deltas
MAGIC = 0x31434642


def seg_header(n, lo, hi):
    """The 16-byte header of a compressed segment: n, hi, lo, magic."""
    return struct.pack("<IIII", n, hi, lo, MAGIC)


def one_segment(ids, lo=0, hi=None):
    ids = np.asarray(ids, np.uint32)
    if hi is None:
        hi = int(ids.max()) + 1
    return Batch(ids, [0, ids.size], [lo], [hi], [0])


def ids_from_deltas(v0, deltas):
    return np.concatenate([[v0], v0 + np.cumsum(deltas)]).astype(np.uint32)


def pfor_size(d, b):
    """Payload words and exception count of a block's deltas d at width b:
    ceil(m b / 32) low words, ceil(E / 4) position words, ceil(E h / 32) high
    words with h = wmin - b when there are exceptions."""
    m = len(d)
    wmin = int(max(d)).bit_length() if m else 0
    E = sum(1 for x in d if int(x) >> b)
    h = wmin - b if E else 0
    return -(-m * b // 32) + -(-E // 4) + -(-E * h // 32), E


def brute_best_b(d):
    wmin = int(max(d)).bit_length() if len(d) else 0
    best = None
    for b in range(wmin + 1):
        w, E = pfor_size(d, b)
        if M10 * E > len(d):
            continue
        if best is None or w <= best[0]:  # ascending b: a tie moves to the larger b
            best = (w, b, E)
    return best


def oracle_pfor(ids):
    d = oracle.block_details(one_segment(ids), [oracle.CLS_PFOR])
    return int(d["words"][0]), int(d["pfor_b"][0]), int(d["pfor_e"][0])


# ------------------------------------------------------------ PFOR width

def test_pfor_width_tie_goes_to_the_larger_width():
    # 31 deltas: 28 of 2 or 3 (two bits) and three of 8..15 (four bits), so
    # wmin = 4.  b = 4: no exception, ceil(31*4/32) = 4 words.  b = 3: three
    # exceptions, 3 + 1 + ceil(3*1/32) = 5 words.  b = 2: the same three
    # exceptions, 2 + 1 + ceil(3*2/32) = 4 words.  b = 1: all 31 deltas are
    # exceptions (31 > 3.1, not allowed).  b = 2 and b = 4 tie at 4 words and
    # the rule keeps b = 4.
    d = [2, 3] * 14 + [9, 12, 15]
    ids = ids_from_deltas(1000, d)
    assert [pfor_size(d, b) for b in (2, 3, 4)] == [(4, 3), (5, 3), (4, 0)]
    assert M10 * pfor_size(d, 1)[1] > len(d)
    assert oracle_pfor(ids) == (4, 4, 0)
    assert brute_best_b(d) == (4, 4, 0)


def test_pfor_width_with_too_many_exceptions_is_not_taken():
    # 31 deltas: 27 of 1 and four of about 2^19 (wmin 20).  Any b in 1..19
    # leaves 4 exceptions (10*4 > 31): not allowed, although b = 1 would need
    # only 1 + 1 + ceil(4*19/32) = 5 words.  Only b = 20 (20 words) is valid.
    d = [1] * 27 + [(1 << 19) + 5, (1 << 19) + 77, (1 << 19) + 1, (1 << 19) + 900]
    ids = ids_from_deltas(7, d)
    assert pfor_size(d, 1) == (5, 4)
    assert oracle_pfor(ids) == (20, 20, 0)


def test_pfor_one_exception_in_ten_is_allowed():
    # 30 deltas, three exceptions: exactly 10 E = m
    d = [1] * 27 + [1 << 12, 1 << 13, 1 << 14]
    w, b, E = oracle_pfor(ids_from_deltas(0, d))
    assert (b, E) == (1, 3)
    assert w == pfor_size(d, 1)[0] == 1 + 1 + -(-3 * 14 // 32)


@pytest.mark.parametrize("seed", range(4))
def test_pfor_width_is_brute_force_minimum(seed):
    rng = np.random.default_rng(100 + seed)
    for t in range(150):
        n = int(rng.choice([2, 5, 17, 31, 64, 100, 127, 128]))
        small = int(rng.integers(1, 6))
        d = rng.integers(1, 1 << small, n - 1)
        nbig = int(rng.integers(0, max(1, (n - 1) // 8)))
        if nbig:
            big = int(rng.integers(small + 1, 27))
            d[rng.choice(n - 1, nbig, replace=False)] = rng.integers(1 << (big - 1), 1 << big, nbig)
        d = [int(x) for x in d]
        w, b, E = oracle_pfor(ids_from_deltas(int(rng.integers(0, 1000)), d))
        assert (w, b, E) == brute_best_b(d), (n, d)


# ------------------------------------------------------------ PFOR layout, every b

def put(bits, pos, width, value):
    for t in range(width):
        if (value >> t) & 1:
            bits[pos + t] = 1


def words_of(bits, nwords):
    out = []
    for k in range(nwords):
        x = 0
        for t in range(32):
            x |= bits[32 * k + t] << t
        out.append(x)
    return out


def pfor_stream(ids, b, lo, hi):
    """One segment holding one PFOR block at width b, assembled field by
    field: low b bits of every delta, exception positions (bytes), high
    parts at h bits."""
    ids = [int(x) for x in ids]
    d = [ids[j] - ids[j - 1] for j in range(1, len(ids))]
    m = len(d)
    wmin = max(d).bit_length() if m else 0
    exc = [j for j in range(m) if d[j] >> b]
    E = len(exc)
    h = wmin - b if E else 0
    lw, qw, hw = -(-m * b // 32), -(-E // 4), -(-E * h // 32)
    low, pos, high = [0] * (32 * lw + 32), [0] * (32 * qw + 32), [0] * (32 * hw + 32)
    for j in range(m):
        put(low, j * b, b, d[j] & ((1 << b) - 1))
    for e, j in enumerate(exc):
        put(pos, 8 * e, 8, j)
        put(high, e * h, h, d[j] >> b)
    payload = words_of(low, lw) + words_of(pos, qw) + words_of(high, hw)
    hdr = seg_header(len(ids), lo, hi)
    entry = struct.pack("<IBBH", ids[0] - lo, oracle.CLS_PFOR, b, E | (h << 8))
    body = hdr + entry + struct.pack("<I", 0) + struct.pack("<%dI" % len(payload), *payload)
    return np.frombuffer(body, np.uint8).copy(), E


def test_every_pfor_width_decodes_from_a_hand_built_stream():
    rng = np.random.default_rng(21)
    seen = set()
    for t in range(60):
        n = int(rng.choice([20, 64, 128]))
        d = rng.integers(1, 1 << int(rng.integers(1, 4)), n - 1)
        k = int(rng.integers(0, (n - 1) // 10 + 1))
        d[rng.choice(n - 1, k, replace=False)] = rng.integers(1 << 8, 1 << int(rng.integers(9, 25)), k)
        ids = ids_from_deltas(int(rng.integers(0, 50)), d)
        lo, hi = 0, int(ids[-1]) + 3
        wmin = int(d.max()).bit_length()
        chosen = oracle_pfor(ids)[1]
        for b in range(wmin + 1):
            stream, E = pfor_stream(ids, b, lo, hi)
            sbo = np.array([0, stream.size], np.uint64)
            st, out, _ = oracle.decode(stream, sbo)
            if M10 * E > n - 1:
                assert st == oracle.ST_CORRUPT
                continue
            assert st == oracle.ST_OK
            np.testing.assert_array_equal(out, ids)
            seen.add(b)
            if b == chosen:
                want, _ = oracle.encode(Batch(ids, [0, n], [lo], [hi]), np.array([oracle.CLS_PFOR], np.uint8),
                                        raw_below=0)
                np.testing.assert_array_equal(stream, want)
    assert seen >= set(range(1, 25))
    # b = 0 leaves every delta (>= 1) an exception, so only a one-ID block
    # (no deltas) can take it
    ids = np.array([77], np.uint32)
    stream, E = pfor_stream(ids, 0, 5, 100)
    st, out, _ = oracle.decode(stream, np.array([0, stream.size], np.uint64))
    assert (st, E) == (oracle.ST_OK, 0)
    np.testing.assert_array_equal(out, ids)


# ------------------------------------------------------------ fp16 rounding points

def diagonal_net(paths):
    """A network in which input i feeds hidden unit i of both layers and
    output class i only: paths[i] = (W1, b1, W2, b2, W3, b3) scalars."""
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(np.zeros(mlp.n_params()))
    W1, b1, W2, b2, W3, b3 = (a.copy() for a in (W1, b1, W2, b2, W3, b3))
    for i, (w1, c1, w2, c2, w3, c3) in enumerate(paths):
        W1[i, i], b1[i], W2[i, i], b2[i], W3[i, i], b3[i] = w1, c1, w2, c2, w3, c3
    return mlp.pack([(W1, b1), (W2, b2), (W3, b3)])


def test_forward_rounds_weights_and_hidden_layers_to_fp16():
    u = 2.0 ** -10  # fp16 spacing in [1, 2); 2u in [2, 4)
    paths = [
        # 0: first-layer weight 1 + 3u/4 rounds to 1 + u; x = 3 gives 3 + 3u,
        #    1.5 spacings above 3: a tie, to even -> 3 + 4u.  Unrounded weight:
        #    3 + 9u/4 -> 3 + 2u.
        (1 + 0.75 * u, 0.0, 1.0, 0.0, 1.0, 0.0),
        # 1: x = 1, bias 2^-11 = u/2: 1 + u/2 is a tie, to even -> h1 = 1; again
        #    in layer 2 -> h2 = 1; logit 1.  Without the first hidden rounding
        #    z2 = 1 + u -> 1 + u; without the second, h2 = 1 + u/2.
        (1.0, 0.5 * u, 1.0, 0.5 * u, 1.0, 0.0),
        # 2: as path 0, in the second layer's weight: 3 + 4u; unrounded 3 + 2u
        (1.0, 0.0, 1 + 0.75 * u, 0.0, 1.0, 0.0),
        # 3: output weight 1 + u/4 rounds to 1; logits are not rounded, so
        #    the output bias 2^-12 = u/4 survives: 1 + u/4.  Unrounded weight:
        #    1 + u/2.
        (1.0, 0.0, 1.0, 0.0, 1 + 0.25 * u, 0.25 * u),
    ]
    theta = diagonal_net(paths)
    X = np.array([[3.0, 1.0, 3.0, 1.0, 0, 0, 0, 0]])
    z, _ = mlp.forward(theta, X)
    want = np.zeros(35)
    want[:4] = [3 + 4 * u, 1.0, 3 + 4 * u, 1 + 0.25 * u]
    np.testing.assert_array_equal(z[0], want)
    # the same values are fp32-exact, so a GPU forward pass has to give them too
    assert (np.float32(want) == want).all()
    # the exact network differs on every path
    ze, _ = mlp.forward(theta, X, rounding=False)
    assert list(ze[0, :4]) == [3 + 2.25 * u, 1 + u, 3 + 2.25 * u, 1 + 0.5 * u]


def test_forward_rounding_of_negative_hidden_values_is_relu_first():
    # ReLU comes before the rounding: a pre-activation of -u/2 gives 0 either
    # way, and a hidden value below the smallest fp16 subnormal (2^-24)
    # rounds to 0: the logit is the output bias alone
    paths = [(1.0, -2.0, 1.0, 0.0, 1.0, 0.5), (2.0 ** -26, 0.0, 1.0, 0.0, 1.0, 0.25)]
    z, _ = mlp.forward(diagonal_net(paths), np.array([[1.0, 1.0, 0, 0, 0, 0, 0, 0]]))
    assert list(z[0, :2]) == [0.5, 0.25]


# ------------------------------------------------------------ compression threshold

def test_raw_form_is_the_ids_verbatim():
    # below the threshold a sequence is sent as it is ("Usage of compression
    # thresholds" section): 4 bytes per ID, no header
    for n in (1, 2, 3, 4, 5, 31):
        ids = np.sort(np.random.default_rng(n).choice(1 << 20, n, replace=False)).astype(np.uint32)
        stream, sbo = oracle.encode(one_segment(ids, hi=1 << 20), raw_below=32)
        assert int(sbo[-1]) == 4 * n
        np.testing.assert_array_equal(stream.view(np.uint32), ids)
        st, out, _ = oracle.decode(stream, sbo)
        assert st == oracle.ST_OK
        np.testing.assert_array_equal(out, ids)


def test_threshold_boundary():
    # n = T - 1 raw, n = T compressed (header n, hi, lo, magic)
    T = 40
    ids = np.arange(100, 100 + 3 * T, 3).astype(np.uint32)
    s1, o1 = oracle.encode(one_segment(ids[:T - 1], hi=1000), raw_below=T)
    s2, o2 = oracle.encode(one_segment(ids[:T], hi=1000), raw_below=T)
    assert int(o1[-1]) == 4 * (T - 1)
    assert struct.unpack("<IIII", s2[:16].tobytes()) == (T, 1000, 0, MAGIC)
    # bit-pack at width 2: 16 + 8 + 4 + ceil(39 * 2 / 32) words
    assert int(o2[-1]) == 16 + 8 + 4 + 4 * 3
    # T = 0 and T = 1 compress every non-empty segment
    for T0 in (0, 1):
        s, o = oracle.encode(one_segment(ids[:1], hi=1000), raw_below=T0)
        assert int(o[-1]) == 28


def test_mixed_batch_offsets_and_round_trip():
    rng = np.random.default_rng(8)
    sizes = [0, 1, 31, 32, 0, 500, 7, 0, 129]
    segs, lo, hi = [], [], []
    base = 0
    for n in sizes:
        segs.append(np.sort(rng.choice(10000, n, replace=False)).astype(np.uint32) + base)
        lo.append(base)
        hi.append(base + 10000)
        base += 10000
    ids = np.concatenate(segs)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    b = Batch(ids, off, lo, hi)
    stream, sbo = oracle.encode(b, raw_below=32)
    lens = np.diff(sbo.astype(np.int64))
    for n, L, s0 in zip(sizes, lens, sbo[:-1]):
        if n == 0:
            assert L == 0
        elif n < 32:
            assert L == 4 * n
        else:
            w = stream[int(s0):int(s0) + 16].view(np.uint32)
            assert w[0] == n and w[1] > w[2] and w[3] == MAGIC
    assert oracle.encoded_size(b, raw_below=32) == int(sbo[-1])
    st, out, oo = oracle.decode(stream, sbo)
    assert st == oracle.ST_OK
    np.testing.assert_array_equal(out, ids)
    np.testing.assert_array_equal(oo, off)
    # the reader needs no threshold: every T gives the same IDs
    for T in (0, 1, 8, 600):
        s, o = oracle.encode(b, raw_below=T)
        st, out, _ = oracle.decode(s, o)
        assert st == oracle.ST_OK
        np.testing.assert_array_equal(out, ids)


def test_single_id_segments_have_ratio_one():
    # a first level of 8 roots split over 16 destinations: 8 one-ID segments
    # and 8 empty ones are 32 bytes, ratio 1 (the compressed form would need
    # 28 bytes per ID)
    roots = np.array([5, 900, 2000, 7000, 9100, 12000, 14500, 16000], np.uint32)
    b = oracle.batch_from_frontier(roots, inputs.bounds_equal(1 << 14, 16))
    stream, sbo = oracle.encode(b)
    assert int(sbo[-1]) == 32
    assert oracle.ratio(4 * roots.size, int(sbo[-1])) == 1.0


def test_reader_rejects_impossible_forms():
    ids = np.arange(10, 50).astype(np.uint32)
    good, sbo = oracle.encode(one_segment(ids, hi=100), raw_below=0)
    # a length that is not a whole number of words
    st, _, _ = oracle.decode(np.concatenate([good, [0]]).astype(np.uint8), np.array([0, good.size + 1], np.uint64))
    assert st == oracle.ST_CORRUPT
    # words 1 and 2 equal: neither form
    s = good.copy().view(np.uint32)
    s[2] = s[1]
    assert oracle.decode(s.view(np.uint8), sbo)[0] == oracle.ST_CORRUPT
    # a compressed header holding no IDs
    s = good.copy().view(np.uint32)
    s[0] = 0
    assert oracle.decode(s.view(np.uint8), sbo)[0] == oracle.ST_CORRUPT
    # raw segments must increase strictly
    for bad in ([5, 5], [9, 3], [1, 2, 3, 3, 4]):
        raw = np.array(bad, np.uint32).view(np.uint8)
        assert oracle.decode(raw, np.array([0, raw.size], np.uint64))[0] == oracle.ST_CORRUPT


def test_default_threshold_gives_ratio_at_least_one_per_level():
    # every BFS level, and every exchanged candidate level, of R-MAT and
    # uniform scale-16 graphs split over 16 equal and 256 Zipf ranges
    for kind in (inputs.RMAT, inputs.UNIFORM):
        g = inputs.graph(kind, 16, 16, 1)
        root = int(inputs.roots(g, 1, 1)[0])
        level, _, depth = oracle.bfs(g, root)
        for bounds in (inputs.bounds_equal(g.n_vertices, 16), inputs.bounds_zipf(g.n_vertices, 256, 1)[0]):
            for L in range(depth + 1):
                f = oracle.frontier(level, L)
                for b in (oracle.batch_from_frontier(f, bounds, L), oracle.candidates(g, f, bounds[::16] if bounds.size > 17 else bounds, L)):
                    stream, sbo = oracle.encode(b)
                    assert oracle.ratio(4 * b.n_ids, int(sbo[-1])) >= 1.0 if b.n_ids else int(sbo[-1]) == 0
