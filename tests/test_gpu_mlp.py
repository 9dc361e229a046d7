"""GPU parity of the learned selector: logits and gradients of the HIP
network against the fp64 oracle (tolerances below), Adam's step, and the
learned class choice resolved and encoded byte-exactly."""
import numpy as np
import pytest

import inputs
import oracle
from oracle import mlp

from gpu_util import gpu_encode, gpu_select, shifted_batch, to_dev, torch

pytestmark = pytest.mark.gpu

# fp32 accumulation of at most 64 fp16 x fp16 products per unit, plus rare
# one-ulp fp16 flips of a hidden value where fp32 and fp64 round differently:
# |dz| <= 2^-11 |h| |w| per flip; the bound below covers a few flips.
LOGIT_RTOL, LOGIT_ATOL = 1e-3, 1e-3
GRAD_RTOL, GRAD_ATOL = 1e-3, 1e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_1704_00513_amd as P
    c = P.Context(0)
    yield c
    c.close()


def frontier_features(n_roots=2):
    g = inputs.graph(inputs.RMAT, 16, 16, 1)
    bs = []
    for root in inputs.roots(g, n_roots, 1):
        level, _, depth = oracle.bfs(g, int(root))
        for L in range(depth + 1):
            bs.append(oracle.batch_from_frontier(oracle.frontier(level, L),
                                                 inputs.bounds_equal(g.n_vertices, 16), L))
    b = oracle.concat_batches(bs)
    return b, oracle.features(b), oracle.select(b)


def test_forward_logits(ctx):
    t = torch()
    b, F, y = frontier_features()
    theta = inputs.mlp_init(3)
    theta[::5] += 0.05
    ctx.mlp_set_weights(theta)
    n = F.shape[0]
    logits = t.zeros((n, 35), dtype=t.float32, device="cuda")
    ctx.mlp_forward(to_dev(F, np.uint16, np.int16), n, logits)
    assert ctx.sync_status() == 0
    got = logits.cpu().numpy()
    want, _ = mlp.forward(theta.astype(np.float64), mlp.features_to_f64(F))
    np.testing.assert_allclose(got, want, rtol=LOGIT_RTOL, atol=LOGIT_ATOL)


@pytest.mark.parametrize("seed", [3, 6])
def test_mfma_inference_matches_oracle(ctx, seed):
    """The matrix-core inference (bfsc_mlp_infer): logits within the same
    tolerance as the vector kernel, and the class equal to the oracle's argmax
    wherever the oracle's top-2 margin is clear of that tolerance.  n is not a
    multiple of 16, so the last group of samples is ragged."""
    t = torch()
    b, F, y = frontier_features()
    F = F[:F.shape[0] - 3]
    theta = inputs.mlp_init(seed)
    theta[::7] += 0.03
    ctx.mlp_set_weights(theta)
    n = F.shape[0]
    assert n % 16 != 0
    logits = t.zeros((n, 35), dtype=t.float32, device="cuda")
    cls = t.zeros(n, dtype=t.uint8, device="cuda")
    ctx.mlp_infer(to_dev(F, np.uint16, np.int16), n, logits, cls)
    assert ctx.sync_status() == 0
    got = logits.cpu().numpy()
    X = mlp.features_to_f64(F)
    want, _ = mlp.forward(theta.astype(np.float64), X)
    np.testing.assert_allclose(got, want, rtol=LOGIT_RTOL, atol=LOGIT_ATOL)
    pred = mlp.predict(theta.astype(np.float64), X)
    top2 = np.sort(want, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * (LOGIT_ATOL + LOGIT_RTOL * np.abs(top2[:, 1]))
    assert clear.mean() > 0.5
    np.testing.assert_array_equal(cls.cpu().numpy()[clear], pred[clear])
    # only the class output requested
    cls2 = t.zeros(n, dtype=t.uint8, device="cuda")
    ctx.mlp_infer(to_dev(F, np.uint16, np.int16), n, None, cls2)
    assert t.equal(cls, cls2)


def test_mfma_inference_nan_weights_give_255(ctx):
    t = torch()
    b, F, y = frontier_features()
    theta = inputs.mlp_init(5)
    theta[-1] = np.nan  # bias of the last class
    ctx.mlp_set_weights(theta)
    n = F.shape[0]
    cls = t.zeros(n, dtype=t.uint8, device="cuda")
    ctx.mlp_infer(to_dev(F, np.uint16, np.int16), n, None, cls)
    assert ctx.sync_status() == 0
    assert (cls.cpu().numpy() == 255).all()
    assert (mlp.predict(theta.astype(np.float64), mlp.features_to_f64(F)) == 255).all()


def test_gradient_matches_oracle(ctx):
    t = torch()
    b, F, y = frontier_features()
    theta = inputs.mlp_init(4)
    ctx.mlp_set_weights(theta)
    n = F.shape[0]
    grads = t.zeros(7011, dtype=t.float32, device="cuda")
    loss = t.zeros(1, dtype=t.float32, device="cuda")
    ctx.mlp_grad(to_dev(F, np.uint16, np.int16), to_dev(y, np.uint8, np.uint8), n, grads, loss)
    assert ctx.sync_status() == 0
    l_ref, g_ref = mlp.loss_and_grad(theta.astype(np.float64), mlp.features_to_f64(F), y)
    assert abs(float(loss.item()) - l_ref) <= 1e-4 * abs(l_ref)
    np.testing.assert_allclose(grads.cpu().numpy(), g_ref, rtol=GRAD_RTOL,
                               atol=GRAD_ATOL * max(1.0, np.abs(g_ref).max()))


def test_adam_steps_match_oracle(ctx):
    # Adam alone, pinned weight by weight: each step's gradient is the GPU's
    # own (bfsc_mlp_grad at the current weights; the gradient kernels reduce
    # in a fixed order, so the training step computes the same vector), fed
    # to the oracle's fp64 Adam from the weights the GPU holds before the
    # step.  What remains is fp32 rounding of the update and the weights.
    t = torch()
    b, F, y = frontier_features()
    theta = inputs.mlp_init(5)
    ctx.mlp_set_weights(theta)
    n = F.shape[0]
    X = to_dev(F, np.uint16, np.int16)
    Y = to_dev(y, np.uint8, np.uint8)
    grads = t.zeros(7011, dtype=t.float32, device="cuda")
    opt = mlp.Adam(theta.size)
    moved = 0
    for step in range(3):
        before = ctx.mlp_get_weights().astype(np.float64)
        ctx.mlp_grad(X, Y, n, grads)
        g = grads.cpu().numpy().astype(np.float64)
        ctx.mlp_train_step(X, Y, n)
        assert ctx.sync_status() == 0
        got = ctx.mlp_get_weights().astype(np.float64)
        want = opt.step(before, g)
        np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-9)
        moved += int(np.sum(got != before))
    assert moved > 3 * 7011 // 2  # most weights move on every step


def test_learned_select_resolves_and_encodes_exactly(ctx):
    b, F, y = frontier_features()
    theta = inputs.mlp_init(6)
    ctx.mlp_set_weights(theta)
    st, got, fb = gpu_select(ctx, b, 2)
    assert st == 0
    # oracle's own prediction, resolved
    z, _ = mlp.forward(theta.astype(np.float64), mlp.features_to_f64(F))
    pred = mlp.predict(theta.astype(np.float64), mlp.features_to_f64(F))
    res, fb_ref = oracle.resolve(b, pred)
    top2 = np.sort(z, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * (LOGIT_ATOL + LOGIT_RTOL * np.abs(top2[:, 1]))
    assert clear.mean() > 0.5
    np.testing.assert_array_equal(got[clear], res[clear])
    # whatever the network picked, the resolved vector is valid and the stream
    # is the oracle's encoding of that vector
    want, want_off = oracle.encode(b, classes=got)
    st, stream, off = gpu_encode(ctx, b, classes=got)
    assert st == 0
    np.testing.assert_array_equal(stream, want)
    np.testing.assert_array_equal(off, want_off)


def test_trained_selector_on_gpu_gains_over_plain(ctx):
    """The committed network on held-out frontiers, run by the GPU kernels:
    its resolved choice encodes byte-exactly, gains over plain packing and
    stays within 2% of exhaustive size."""
    import os
    from test_selector_trained import WEIGHTS, held_out_batches
    if not os.path.exists(WEIGHTS):
        pytest.skip("selector not trained")
    ctx.mlp_set_weights(np.load(WEIGHTS, allow_pickle=False))
    plain = exh = learned = 0
    for b in held_out_batches():
        print("trained selector n=%d nseg=%d" % (b.n_ids, b.nseg), flush=True)
        st, cls, fb = gpu_select(ctx, b, 2)
        assert st == 0
        want, want_off = oracle.encode(b, classes=cls)
        st, stream, off = gpu_encode(ctx, b, classes=cls)
        assert st == 0
        np.testing.assert_array_equal(stream, want)
        np.testing.assert_array_equal(off, want_off)
        learned += stream.size
        plain += oracle.encode(b, mode=oracle.PLAIN_BP)[0].size
        exh += oracle.encode(b, mode=oracle.EXHAUSTIVE)[0].size
    assert learned <= 0.85 * plain, (learned, plain)
    assert learned <= 1.02 * exh, (learned, exh)


def _codec_batches():
    from test_gpu_codec import batches
    return [b for name, b in batches()] + [b for b in _held_out()]


def _held_out():
    from test_selector_trained import held_out_batches
    return held_out_batches()


@pytest.mark.parametrize("weights", ["random", "trained"])
@pytest.mark.parametrize("waves,strided", [(4, 1), (4, 0), (1, 1), (2, 1), (8, 1)])
def test_fused_learned_encode_equals_two_pass(ctx, weights, waves, strided):
    """bfsc_encode with the learned mode and no class vector (the network
    inside the pack pass) writes the same bytes as bfsc_select + bfsc_encode,
    and those are the oracle's encoding of the selected classes.  Random
    weights reach every resolve branch, fallbacks included."""
    import os
    from test_selector_trained import WEIGHTS
    if weights == "trained":
        if not os.path.exists(WEIGHTS):
            pytest.skip("selector not trained")
        theta = np.load(WEIGHTS, allow_pickle=False)
    else:
        theta = inputs.mlp_init(11)
        theta[::3] *= 4.0
    ctx.mlp_set_weights(theta)
    before = ctx.get_tune()
    ctx.set_tune(enc_waves=waves, enc_pack=4 * strided)
    try:
        seen = set()
        for b in _codec_batches():
            print("fused learned n=%d nseg=%d" % (b.n_ids, b.nseg), flush=True)
            st, cls, fb = gpu_select(ctx, b, 2)
            assert st == 0
            seen.update(np.unique(cls).tolist())
            st, two, two_off = gpu_encode(ctx, b, classes=cls)
            assert st == 0
            st, fused, fused_off = gpu_encode(ctx, b, mode=2)
            assert st == 0
            np.testing.assert_array_equal(fused_off, two_off)
            np.testing.assert_array_equal(fused, two)
            want, want_off = oracle.encode(b, classes=cls)
            np.testing.assert_array_equal(fused, want)
        if weights == "random":
            assert len(seen) >= 2
    finally:
        ctx.set_tune(**before)


def test_fused_learned_unaligned_ids(ctx):
    """The fused learned pack pass reading IDs that are not 16-byte aligned
    (its row path loads them word by word) writes the oracle's encoding of
    the selected classes."""
    import paper_1704_00513_amd as P
    theta = inputs.mlp_init(11)
    theta[::3] *= 4.0
    ctx.mlp_set_weights(theta)
    t = torch()
    for b in _codec_batches():
        if b.n_ids < 1024:
            continue
        st, cls, _ = gpu_select(ctx, b, 2)
        assert st == 0
        want, want_off = oracle.encode(b, classes=cls)
        for shift in (1, 3):
            print("fused learned unaligned shift=%d n=%d" % (shift, b.n_ids), flush=True)
            db, keep = shifted_batch(b, shift)
            cap = P.Context.encode_bound(b.n_ids, b.nseg)
            out = t.zeros(cap, dtype=t.uint8, device="cuda")
            sbo = t.zeros(b.nseg + 1, dtype=t.int64, device="cuda")
            ctx.encode(db, out, sbo, mode=2, out_cap=cap)
            assert ctx.sync_status() == 0
            sbo_h = sbo.cpu().numpy().view(np.uint64)
            np.testing.assert_array_equal(sbo_h, want_off)
            np.testing.assert_array_equal(out[:int(sbo_h[-1])].cpu().numpy(), want)
            del keep
