"""Pins for the oracle's learned-tagger network (a project addition, not in
the paper): finite-difference gradients, known answers of the convolution,
and BF16 rounding."""
import numpy as np
import pytest

import oracle

NIN = 13


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(oracle.cnn_num_params(NIN)) * scale


def test_parameter_count():
    # 3x3 convs 13->32->32->32 with biases, head 32->3 with bias
    assert oracle.cnn_num_params(NIN) == 32 * 13 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 3 * 32 + 3


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params(2)
    x = rng.standard_normal((3, NIN, 16, 16))
    labels = np.array([0, 2, 1])
    loss, g = oracle.cnn_grad(p, x, labels)
    idx = rng.choice(len(p), 60, replace=False)
    n = oracle.cnn_num_params(NIN)
    # include head, biases and first-layer weights explicitly
    idx = np.unique(np.concatenate([idx, [0, 5, 32 * 13 * 9 + 3, n - 1, n - 50]]))
    h = 1e-5
    for i in idx:
        pp = p.copy(); pp[i] += h
        lp = oracle.cnn_forward(pp, x, labels)[1]
        pp[i] -= 2 * h
        lm = oracle.cnn_forward(pp, x, labels)[1]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])


def test_identity_kernel_and_padding():
    """A layer whose kernel is a centred delta copies its input; a delta at
    (ky,kx)=(0,0) shifts by one pixel with zero padding; the pooled mean of a
    constant image is that constant."""
    n = oracle.cnn_num_params(NIN)
    p = np.zeros(n)
    # layer 1: channel 0 <- input channel 4 (centre tap); layers 2, 3 identity on channel 0
    o1 = 0
    p[o1 + ((0 * NIN + 4) * 3 + 1) * 3 + 1] = 1.0
    o2 = 32 * NIN * 9 + 32
    p[o2 + ((0 * 32 + 0) * 3 + 1) * 3 + 1] = 1.0
    o3 = o2 + 32 * 32 * 9 + 32
    p[o3 + ((0 * 32 + 0) * 3 + 0) * 3 + 0] = 1.0  # shift: out(y,x) = in(y-1,x-1)
    oh = o3 + 32 * 32 * 9 + 32
    p[oh + 2 * 32 + 0] = 1.0  # refine logit = pooled channel 0
    x = np.zeros((1, NIN, 16, 16))
    x[0, 4] = np.arange(256).reshape(16, 16) / 256.0
    logits, _ = oracle.cnn_forward(p, x)
    shifted = np.zeros((16, 16))
    shifted[1:, 1:] = x[0, 4][:-1, :-1]
    assert abs(logits[0, 2] - shifted.mean()) < 1e-15
    assert abs(logits[0, 0]) < 1e-15 and abs(logits[0, 1]) < 1e-15


def test_bf16_rounding_is_round_to_nearest_even():
    assert oracle.round_bf16(1.0) == 1.0
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even (1.0)
    assert oracle.round_bf16(1.0 + 2 ** -8) == 1.0
    assert oracle.round_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert oracle.round_bf16(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    assert oracle.round_bf16(-3.0e38) < -3.0e38 * 0.99


def test_bf16_forward_close_to_fp64():
    rng = np.random.default_rng(3)
    p = _params(4, 0.2)
    x = rng.standard_normal((2, NIN, 16, 16))
    l64, _ = oracle.cnn_forward(p, x)
    l16, _ = oracle.cnn_forward(p, x, bf16=True)
    assert np.abs(l16 - l64).max() < 0.05 * max(1.0, np.abs(l64).max())
    assert np.abs(l16 - l64).max() > 0.0
