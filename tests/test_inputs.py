"""The seeded input generators: determinism, graph hygiene, R-MAT quadrant
frequencies and the Zipf sampler against its exact probability mass."""
import hashlib
import json
import os

import numpy as np
import pytest
from scipy import stats

import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "inputs_hashes.json")


def graph_hash(g):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g.row_ptr).tobytes())
    h.update(np.ascontiguousarray(g.col_idx).tobytes())
    return h.hexdigest()


def test_generator_is_deterministic_and_matches_golden():
    with open(GOLDEN) as f:
        gold = json.load(f)
    for key, want in gold["graphs"].items():
        kind, scale, seed = key.split("-")
        g = inputs.Graph(inputs.RMAT if kind == "rmat" else inputs.UNIFORM, int(scale), 16,
                         int(seed))
        assert graph_hash(g) == want, key
    g = inputs.graph(inputs.RMAT, 16, 16, 1)
    assert [int(x) for x in inputs.roots(g, 8, 1)] == gold["roots_s16_seed1"]


@pytest.mark.parametrize("kind", [inputs.RMAT, inputs.UNIFORM])
def test_csr_is_symmetric_simple_and_sorted(kind):
    g = inputs.graph(kind, 12, 16, 2)
    V = g.n_vertices
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.n_arcs
    src = np.repeat(np.arange(V, dtype=np.int64), np.diff(g.row_ptr).astype(np.int64))
    dst = g.col_idx.astype(np.int64)
    assert not np.any(src == dst)  # no self-loops
    key = src * V + dst
    assert np.all(np.diff(key) > 0)  # rows ascending, no duplicates
    rkey = np.sort(dst * V + src)
    np.testing.assert_array_equal(key, rkey)  # symmetric
    # every arc comes from a sample: at most 2 arcs per sample
    assert g.n_arcs <= 2 * 16 * V


def test_rmat_quadrant_frequencies():
    u, v = inputs.samples(inputs.RMAT, 20, 1, 0, 400000)
    top = 1 << 19
    q = (u >= top).astype(int) * 2 + (v >= top).astype(int)  # 0=a, 1=b, 2=c, 3=d
    counts = np.bincount(q, minlength=4)
    expect = np.array([0.57, 0.19, 0.19, 0.05]) * u.size
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < stats.chi2.ppf(0.9999, 3)
    # lower bit levels follow the same law
    q2 = ((u >> 3) & 1) * 2 + ((v >> 3) & 1)
    counts = np.bincount(q2, minlength=4)
    assert ((counts - expect) ** 2 / expect).sum() < stats.chi2.ppf(0.9999, 3)


def test_uniform_samples_are_uniform():
    u, v = inputs.samples(inputs.UNIFORM, 12, 1, 0, 200000)
    counts = np.bincount(u >> 6, minlength=64)
    expect = u.size / 64
    assert ((counts - expect) ** 2 / expect).sum() < stats.chi2.ppf(0.9999, 63)


def test_zipf_draws_follow_exact_pmf():
    s, kmax = 1.2, 1 << 20
    x = inputs.zipf_draws(1_000_000, 5, s, kmax)
    assert x.min() >= 1 and x.max() <= kmax
    k = np.arange(1, kmax + 1, dtype=np.float64)
    pmf = k ** -s
    pmf /= pmf.sum()
    edges = [1, 2, 3, 4, 5, 7, 10, 20, 50, 100, 1000, 10000, kmax + 1]
    obs = np.array([((x >= a) & (x < b)).sum() for a, b in zip(edges[:-1], edges[1:])])
    cdf = np.concatenate([[0], np.cumsum(pmf)])
    exp = np.array([cdf[b - 1] - cdf[a - 1] for a, b in zip(edges[:-1], edges[1:])]) * x.size
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < stats.chi2.ppf(0.9999, len(obs) - 1)


def test_bounds():
    b = inputs.bounds_equal(1 << 22, 16)
    assert b[0] == 0 and b[-1] == 1 << 22 and np.all(np.diff(b.astype(np.int64)) == 1 << 18)
    z, ks = inputs.bounds_zipf(1 << 24, 256, 1)
    assert z[0] == 0 and z[-1] == 1 << 24 and np.all(np.diff(z.astype(np.int64)) >= 0)
    # proportional to the draws
    widths = np.diff(z.astype(np.float64))
    np.testing.assert_allclose(widths / widths.sum(), ks / ks.sum(), atol=2.0 / (1 << 24) * 256)


def test_roots_are_distinct_and_not_isolated():
    g = inputs.graph(inputs.RMAT, 14, 16, 3)
    r = inputs.roots(g, 16, 3)
    assert r.size == 16 and np.unique(r).size == 16
    assert np.all(np.diff(g.row_ptr)[r] > 0)


def test_mlp_init_is_he_uniform():
    w = inputs.mlp_init(1)
    assert w.size == inputs.mlp_param_count() == 8 * 64 + 64 + 64 * 64 + 64 + 64 * 35 + 35
    W1 = w[:512]
    assert np.abs(W1).max() <= np.sqrt(6 / 8) and np.abs(W1).max() > 0.8 * np.sqrt(6 / 8)
    assert np.all(w[512:576] == 0)
