"""Pins of the learned-selector oracle: fp16 conversion against numpy's IEEE
conversion, features on blocks with hand-derived values, the MLP backward
pass against finite differences, closed forms of the loss and of Adam's first
step, and the resolve rules."""
import numpy as np
import pytest

import inputs
import oracle
from oracle import Batch
from oracle import mlp


def test_f32_to_f16_matches_numpy_ieee_conversion():
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.standard_normal(20000).astype(np.float32),
        (rng.random(20000) * 2.0 ** rng.integers(-30, 20, 20000)).astype(np.float32),
        np.array([0.0, -0.0, 1.0, 65504.0, 65520.0, 65519.99, 1e-8, 6.1e-5, 5.96e-8, 2.98e-8,
                  np.inf, -np.inf, 1 / 3, 2049.0, 2051.0, 0.1], np.float32),
    ])
    # exact ties in binary16 rounding: 1 + (2k+1) * 2^-11
    ties = (1.0 + (2 * np.arange(100) + 1) * 2.0 ** -11).astype(np.float32)
    vals = np.concatenate([vals, ties, -ties])
    with np.errstate(over="ignore"):
        want = vals.astype(np.float16).view(np.uint16)
    got = np.array([oracle.f32_to_f16(v) for v in vals], np.uint16)
    np.testing.assert_array_equal(got, want)


def test_features_of_hand_made_blocks():
    f16 = lambda x: int(np.float16(x).view(np.uint16))
    # 128 consecutive IDs, level 5, segment of 300 IDs
    ids = np.concatenate([np.arange(1000, 1128), np.arange(5000, 5000 + 172 * 3, 3)]).astype(np.uint32)
    b = Batch(ids, [0, ids.size], [0], [1 << 20], [5])
    F = oracle.features(b)
    assert F.shape == (3, 8)
    # block 0: n=128, all gaps 1, span 127
    want0 = [1.0, 1 / 32, 1 / 32, 1 / 32, 7 / 32, 128 / 128, 5 / 64, 9 / 32]
    assert list(F[0]) == [f16(x) for x in want0]
    # block 1: 1127 -> 5000 then 127 gaps... first value 5000+? (IDs 128..255)
    blk = ids[128:256].astype(np.int64)
    d = np.diff(blk)
    span = blk[-1] - blk[0]
    want1 = [1.0, int(d.min()).bit_length() / 32, int(d.max()).bit_length() / 32,
             int(span // 127).bit_length() / 32, int(span).bit_length() / 32,
             np.float32(128) / np.float32(span + 1), 5 / 64, 9 / 32]
    assert list(F[1]) == [f16(x) for x in want1]
    # block 2: 300 - 256 = 44 IDs, gaps 3
    want2 = [44 / 128, 2 / 32, 2 / 32, 2 / 32, int(43 * 3).bit_length() / 32,
             np.float32(44) / np.float32(43 * 3 + 1), 5 / 64, 9 / 32]
    assert list(F[2]) == [f16(x) for x in want2]


def test_features_single_id_and_level_clamp():
    b = Batch(np.array([7], np.uint32), [0, 1], [0], [8], [200])
    F = oracle.features(b)[0].view(np.float16).astype(np.float64)
    assert list(F) == [1 / 128, 0, 0, 0, 0, 1.0, 63 / 64, 1 / 32]


# ------------------------------------------------------------------ MLP

def small_problem(n=64, seed=0):
    rng = np.random.default_rng(seed)
    X = mlp.f16(rng.random((n, 8)))
    y = rng.integers(0, 35, n)
    theta = inputs.mlp_init(seed + 1).astype(np.float64)
    theta[np.arange(theta.size) % 7 == 0] += 0.01  # nonzero biases too
    return theta, X, y


def test_backward_matches_finite_differences():
    theta, X, y = small_problem()
    loss, g = mlp.loss_and_grad(theta, X, y, rounding=False)
    rng = np.random.default_rng(1)
    idx = rng.choice(theta.size, 60, replace=False)
    fd = mlp.finite_difference(theta, X, y, idx)
    np.testing.assert_allclose(g[idx], fd, rtol=1e-6, atol=1e-9)


def test_straight_through_equals_exact_when_rounding_is_exact():
    # weights and inputs on a coarse dyadic grid: every fp16 rounding is the
    # identity, so the rounded network equals the exact one
    rng = np.random.default_rng(2)
    theta = rng.integers(-1, 2, mlp.n_params()) * (rng.random(mlp.n_params()) < 0.2) / 4.0
    X = rng.integers(0, 2, (32, 8)).astype(np.float64)
    y = rng.integers(0, 35, 32)
    z_r, _ = mlp.forward(theta, X, True)
    z_e, _ = mlp.forward(theta, X, False)
    # hidden values are sums of few dyadic terms: exact in fp16 while small
    np.testing.assert_array_equal(z_r, z_e)
    l1, g1 = mlp.loss_and_grad(theta, X, y, True)
    l2, g2 = mlp.loss_and_grad(theta, X, y, False)
    np.testing.assert_array_equal(g1, g2)


def test_zero_network_loss_is_log_35():
    theta = np.zeros(mlp.n_params())
    X = np.ones((10, 8))
    loss, g = mlp.loss_and_grad(theta, X, np.arange(10) % 35)
    assert loss == pytest.approx(np.log(35.0))
    # with zero weights only the output bias gets a gradient: mean(p - onehot)
    (dW1, db1), (dW2, db2), (dW3, db3) = mlp.unpack(g)
    assert not dW1.any() and not dW2.any() and not dW3.any()
    want = np.full(35, 1 / 35.0)
    want -= np.bincount(np.arange(10) % 35, minlength=35) / 10.0
    np.testing.assert_allclose(db3, want, atol=1e-15)


def test_logits_are_output_bias_for_zero_hidden():
    theta = np.zeros(mlp.n_params())
    (_, _), (_, _), (_, b3) = mlp.unpack(theta)
    theta[-35:] = np.arange(35) * 0.5
    z, _ = mlp.forward(theta, np.ones((3, 8)))
    np.testing.assert_array_equal(z, np.tile(np.arange(35) * 0.5, (3, 1)))


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(3)
    g = rng.standard_normal(100)
    theta = rng.standard_normal(100)
    opt = mlp.Adam(100, lr=1e-3)
    new = opt.step(theta, g)
    # m_hat = g, v_hat = g^2 after bias correction -> step = lr g / (|g| + eps)
    np.testing.assert_allclose(theta - new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_predict_ties_and_nan():
    theta = np.zeros(mlp.n_params())
    X = np.ones((2, 8))
    assert list(mlp.predict(theta, X)) == [0, 0]  # all-equal logits -> lowest index
    theta[-35:] = np.nan
    assert list(mlp.predict(theta, X)) == [255, 255]


# ------------------------------------------------------------------ resolve

def test_resolve_rules():
    # block A: 128 IDs with span > 4096 (bitmap invalid); block B: dense
    a = np.arange(128, dtype=np.int64) * 100
    bb = 20000 + np.arange(128, dtype=np.int64)
    ids = np.concatenate([a, bb]).astype(np.uint32)
    b = Batch(ids, [0, 256], [0], [1 << 20])
    ex = oracle.select(b)
    wminA = int(99).bit_length()  # gaps of 100 -> 7 bits
    # bitmap on A falls back to exhaustive; bitmap on B stays
    res, fb = oracle.resolve(b, np.array([0, 0], np.uint8))
    assert list(res) == [ex[0], 0] and fb == 1
    # any BP class snaps to the minimal width
    res, fb = oracle.resolve(b, np.array([33, 5], np.uint8))
    assert list(res) == [1 + wminA, 2] and fb == 0
    # literal: too narrow falls back; wide enough stays
    res, fb = oracle.resolve(b, np.array([3, 9], np.uint8), literal=True)
    assert list(res) == [ex[0], 9] and fb == 1
    # PFOR kept; out-of-range prediction falls back
    res, fb = oracle.resolve(b, np.array([34, 255], np.uint8))
    assert list(res) == [34, ex[1]] and fb == 1
    # every resolved vector encodes and decodes losslessly
    for pred in ([0, 0], [33, 5], [34, 34], [255, 255]):
        res, _ = oracle.resolve(b, np.array(pred, np.uint8))
        stream, sbo = oracle.encode(b, res)
        st, out, _ = oracle.decode(stream, sbo)
        assert st == 0 and np.array_equal(out, ids)
