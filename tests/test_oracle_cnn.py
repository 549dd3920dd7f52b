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


def test_conv_backward_is_the_adjoint():
    """The per-layer backward is the adjoint of the convolution: with
    y = conv(x, w) (no bias), <dz, y> = <dx, x> = <gW, w>, and the bias
    gradient is the pixel sum of dz (exact identities of a bilinear map)."""
    rng = np.random.default_rng(21)
    B, cin = 2, 5
    x = rng.standard_normal((B, cin, 16, 16))
    w = rng.standard_normal((32, cin, 3, 3))
    dz = rng.standard_normal((B, 32, 16, 16))
    y = oracle.cnn_conv(x, w, np.zeros(32))
    gW, gb, dx = oracle.cnn_conv_backward(x, w, dz)
    lhs = float((dz * y).sum())
    assert abs(lhs - float((dx * x).sum())) <= 1e-10 * abs(lhs)
    assert abs(lhs - float((gW * w).sum())) <= 1e-10 * abs(lhs)
    np.testing.assert_allclose(gb, dz.sum(axis=(0, 2, 3)), rtol=1e-13)


@pytest.mark.parametrize("bf16", [False, True])
def test_layerwise_backward_composes_to_the_gradient(bf16):
    """Head and per-layer backward, chained by hand through the ReLUs, give
    the whole-network gradient (itself pinned by finite differences above)."""
    rng = np.random.default_rng(22)
    nin, B = 13, 3
    p = rng.standard_normal(oracle.cnn_num_params(nin)) * 0.3
    x = rng.standard_normal((B, nin, 16, 16))
    labels = np.array([2, 0, 1], np.int32)
    loss, g = oracle.cnn_grad(p, x, labels, bf16=bf16)
    sl, o = [], 0
    for cin in (nin, 32, 32):
        sl.append((o, o + 32 * cin * 9, o + 32 * cin * 9 + 32, cin))
        o += 32 * cin * 9 + 32
    # forward by layers
    a, zs, ins = x, [], []
    for (w0, w1, b1, cin) in sl:
        ins.append(a)
        z = oracle.cnn_conv(a, p[w0:w1].reshape(32, cin, 3, 3), p[w1:b1], bf16=bf16)
        zs.append(z)
        a = np.maximum(z, 0.0)
    loss2, _, gWh, gbh, da = oracle.cnn_head(p, a, labels)
    assert abs(loss2 - loss) <= 1e-12 * abs(loss)
    np.testing.assert_allclose(gWh.ravel(), g[o:o + 96], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gbh, g[o + 96:o + 99], rtol=1e-12, atol=1e-15)
    for l in (2, 1, 0):
        w0, w1, b1, cin = sl[l]
        dz = np.where(zs[l] > 0.0, da, 0.0)
        gW, gb, da = oracle.cnn_conv_backward(ins[l], p[w0:w1].reshape(32, cin, 3, 3), dz, bf16=bf16)
        np.testing.assert_allclose(gW.ravel(), g[w0:w1], rtol=1e-11, atol=1e-14 * np.abs(g[w0:w1]).max())
        np.testing.assert_allclose(gb, g[w1:b1], rtol=1e-11, atol=1e-14 * np.abs(g[w1:b1]).max())
