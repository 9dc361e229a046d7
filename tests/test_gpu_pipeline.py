"""GPU parity of the per-level pipeline (BFS level -> partition -> choose ->
encode -> decode), replayed from captured HIP graphs and launched eagerly:
every level of every replay is checked against the oracle, with host work
and synchronisation between replays; and the autotuner's choice keeps the
streams byte-exact."""
import numpy as np
import pytest

import inputs
import oracle

from gpu_util import gpu_encode, stream_classes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


def run_pipeline(ctx, g, root, bounds, use_graph, mode=1, theta=None):
    """theta: the network's weights in learned mode (mode 2): each level's
    stream must then be the oracle's encoding of the classes its directory
    records, and those must be the oracle's resolved prediction wherever its
    top two logits are clearly apart."""
    import paper_1704_00513_amd as P
    from oracle import mlp
    dg = P.DeviceGraph.from_host(g)
    pipe = P.Pipeline(ctx, dg, bounds, mode=mode, use_graph=use_graph)
    olevel, _, depth = oracle.bfs(g, root)
    checked = 0
    pipe.start(root)
    L = 0
    n = 1
    while n:
        n = pipe.step()
        assert ctx.sync_status() == 0
        got = pipe.last_step()
        front = oracle.frontier(olevel, L)
        np.testing.assert_array_equal(got["frontier"], front)
        ob = oracle.batch_from_frontier(front, bounds, L)
        np.testing.assert_array_equal(got["seg_off"], ob.seg_off)
        if mode == 2:
            cls = stream_classes(got["stream"], got["seg_byte_off"], ob.seg_off)
            want, want_off = oracle.encode(ob, classes=cls)
            X = mlp.features_to_f64(oracle.features(ob))
            z, _ = mlp.forward(theta, X)
            res, _ = oracle.resolve(ob, mlp.predict(theta, X))
            top2 = np.sort(z, axis=1)[:, -2:]
            clear = (top2[:, 1] - top2[:, 0]) > 2e-3 * (1 + np.abs(top2[:, 1]))
            sizes = np.diff(ob.seg_off.astype(np.int64))
            comp = np.repeat(sizes >= oracle.RAW_BELOW, (sizes + 127) // 128)
            np.testing.assert_array_equal(cls[clear & comp], res[clear & comp])
            checked += int((clear & comp).sum())
        else:
            want, want_off = oracle.encode(ob, mode=mode)
        np.testing.assert_array_equal(got["seg_byte_off"], want_off)
        np.testing.assert_array_equal(got["stream"], want)
        np.testing.assert_array_equal(got["decoded"], front)
        np.testing.assert_array_equal(got["decoded_off"], ob.seg_off)
        L += 1
        assert L <= depth + 1
    assert L == depth + 1
    lv, par = pipe.levels()
    np.testing.assert_array_equal(lv, olevel)
    assert oracle.bfs_check(g, root, lv, par) == 0
    pipe.close()
    if mode == 2:
        assert checked > 0
    return L


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("kind,scale,nseg,zipf", [(inputs.RMAT, 14, 16, False),
                                                  (inputs.RMAT, 16, 64, True),
                                                  (inputs.UNIFORM, 15, 16, False)])
def test_pipeline_levels_exact(ctx, use_graph, kind, scale, nseg, zipf):
    g = inputs.graph(kind, scale, 16, 1)
    bounds = inputs.bounds_zipf(g.n_vertices, nseg, 1)[0] if zipf else inputs.bounds_equal(g.n_vertices, nseg)
    for root in inputs.roots(g, 2, 1):
        print("pipeline graph=%s kind=%d scale=%d nseg=%d root=%d" % (use_graph, kind, scale, nseg, root),
              flush=True)
        run_pipeline(ctx, g, int(root), bounds, use_graph)


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("alpha,beta", [(14.0, 24.0), (1e9, 1e9)])
def test_pipeline_direction_optimizing(ctx, use_graph, alpha, beta):
    """Direction-optimizing levels inside the captured pipeline: the
    direction is decided on the device at every replay."""
    g = inputs.graph(inputs.RMAT, 15, 16, 3)
    ctx.bfs_set_direction(alpha, beta)
    try:
        for root in inputs.roots(g, 2, 3):
            print("pipeline-do graph=%s alpha=%g root=%d" % (use_graph, alpha, root), flush=True)
            run_pipeline(ctx, g, int(root), inputs.bounds_equal(g.n_vertices, 16), use_graph)
    finally:
        ctx.bfs_set_direction(0.0, 0.0)


@pytest.mark.parametrize("use_graph", [True, False])
def test_pipeline_learned_mode(ctx, use_graph):
    """The learned choice inside the captured level (fused into the pack
    pass), with the trained selector."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1704_00513_amd", "selector_weights.npy")
    theta = np.load(path, allow_pickle=False)
    ctx.mlp_set_weights(theta)
    g = inputs.graph(inputs.RMAT, 16, 16, 1)
    bounds = inputs.bounds_zipf(g.n_vertices, 64, 1)[0]
    for root in inputs.roots(g, 2, 1):
        print("pipeline learned graph=%s root=%d" % (use_graph, root), flush=True)
        run_pipeline(ctx, g, int(root), bounds, use_graph, mode=2, theta=theta.astype(np.float64))


def test_pipeline_plain_mode(ctx):
    g = inputs.graph(inputs.RMAT, 14, 16, 2)
    root = int(inputs.roots(g, 1, 2)[0])
    print("pipeline plain", flush=True)
    run_pipeline(ctx, g, root, np.array([0, g.n_vertices], np.uint32), True, mode=0)


def test_autotune_keeps_streams_exact(ctx):
    import paper_1704_00513_amd as P
    from gpu_util import device_batch
    g = inputs.graph(inputs.RMAT, 16, 16, 1)
    level, _, depth = oracle.bfs(g, int(inputs.roots(g, 1, 1)[0]))
    bs = [oracle.batch_from_frontier(oracle.frontier(level, L), inputs.bounds_equal(g.n_vertices, 16), L)
          for L in range(depth + 1)]
    b = oracle.concat_batches(bs)
    before = ctx.get_tune()
    tuned = ctx.autotune(device_batch(b))
    print("autotune", before, "->", tuned, flush=True)
    assert tuned["enc_waves"] in (1, 2, 4, 8, 16) and tuned["dec_waves"] in (1, 2, 4, 8, 16)
    want, want_off = oracle.encode(b)
    st, got, off = gpu_encode(ctx, b)
    assert st == 0
    np.testing.assert_array_equal(got, want)
    ctx.set_tune(**before)
