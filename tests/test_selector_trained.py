"""The trained selector (paper_1704_00513_amd/selector_weights.npy), judged on
frontiers of a graph it was not trained on (R-MAT scale 16, seed 9; training
used seeds 1..5): what it gains over plain minimal-width bit-packing, and how
far it stays from the exhaustive choice.  CPU only: the oracle's fp64 forward
pass of the network, resolved and encoded by the oracle."""
import os

import numpy as np
import pytest

import inputs
import oracle
from oracle import mlp

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_1704_00513_amd", "selector_weights.npy")


def held_out_batches(scale=16, seed=9):
    g = inputs.graph(inputs.RMAT, scale, 16, seed)
    root = int(inputs.roots(g, 1, seed)[0])
    level, _, depth = oracle.bfs(g, root)
    out = []
    for bounds in (inputs.bounds_equal(g.n_vertices, 16), inputs.bounds_zipf(g.n_vertices, 256, seed)[0]):
        for L in range(depth + 1):
            b = oracle.batch_from_frontier(oracle.frontier(level, L), bounds, L)
            if b.n_ids:
                out.append(b)
    return out


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="selector not trained")
def test_trained_selector_gain_and_gap():
    theta = np.load(WEIGHTS, allow_pickle=False).astype(np.float64)
    assert theta.size == mlp.n_params()
    plain = exh = learned = fallbacks = blocks = 0
    for b in held_out_batches():
        pred = mlp.predict(theta, mlp.features_to_f64(oracle.features(b)))
        res, fb = oracle.resolve(b, pred)
        stream, sbo = oracle.encode(b, classes=res)
        st, ids, _ = oracle.decode(stream, sbo)
        assert st == 0 and np.array_equal(ids, b.ids)
        learned += stream.size
        plain += oracle.encode(b, mode=oracle.PLAIN_BP)[0].size
        exh += oracle.encode(b, mode=oracle.EXHAUSTIVE)[0].size
        fallbacks += fb
        blocks += b.n_blocks
    # the network buys most of what exhaustive search buys over plain packing
    assert learned <= 0.85 * plain, (learned, plain)
    # and stays within 2% of the exhaustive size
    assert learned <= 1.02 * exh, (learned, exh)
    assert fallbacks <= 0.01 * blocks
