"""Learned tagger on the GPU (BF16 matrix-core convolutions, FP32
accumulation) against the FP64 oracle network with BF16 operand rounding."""
import os

import numpy as np
import pytest

import afsynth
import oracle
import paper_2205_07572_amd as af

pytestmark = pytest.mark.gpu
NIN = 13


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU on this machine")
    assert torch.cuda.is_available(), "GPU present but torch.cuda.is_available() is False"


def _bf16(a):
    """Round to FP32 then to BF16 (nearest even), as both implementations do."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _slices(nin=NIN):
    o, out = 0, {}
    for l, cin in enumerate([nin, 32, 32]):
        out[f"W{l}"] = (o, o + 32 * cin * 9, (32, cin, 3, 3)); o += 32 * cin * 9
        out[f"b{l}"] = (o, o + 32, (32,)); o += 32
    out["Wh"] = (o, o + 96, (3, 32)); o += 96
    out["bh"] = (o, o + 3, (3,)); o += 3
    return out


def _get(p, name):
    a, b, shape = _slices()[name]
    return p[a:b].reshape(shape)


def _setup(seed, B=5, scale=0.25):
    import torch
    rng = np.random.default_rng(seed)
    t = af.Tagger(NIN)
    p = (rng.standard_normal(t.nparams) * scale).astype(np.float32)
    t.set_params(p)
    x = rng.standard_normal((B, NIN, 16, 16)).astype(np.float32)
    return t, p.astype(np.float64), x, torch.from_numpy(x).cuda()


U32 = 2.0 ** -24  # unit roundoff of FP32


def _nhwc(a, B):
    """[3][B*256][32] (pixel-major, channel-minor) -> [3][B][32][16][16]."""
    return a.cpu().numpy().astype(np.float64).reshape(3, B, 16, 16, 32).transpose(0, 1, 4, 2, 3)


def _check(name, got, ref, bound):
    err = np.abs(np.asarray(got, np.float64) - ref)
    ratio = float((err / np.maximum(bound, 1e-300)).max())
    print(f"[gpu-cnn] {name}: max |err| / bound = {ratio:.3f}", flush=True)
    assert (err <= bound).all(), (name, ratio)


def test_layer_by_layer_parity():
    """Each layer's pre-activation equals the oracle's convolution of the same
    BF16 operands to FP32 accumulation accuracy, entry by entry:
    |err| <= sqrt(K) 2^-24 sum |a w| over the K <= 288 products, plus one
    rounding of the bias addition."""
    import torch
    t, p, x, xd = _setup(1)
    B = x.shape[0]
    logits, acts = t.forward(xd, acts=True)
    torch.cuda.synchronize()
    acts = _nhwc(acts, B)
    inp = x.astype(np.float64)
    for l in range(3):
        W, b = _get(p, f"W{l}"), _get(p, f"b{l}")
        K = 9 * W.shape[1]
        ref = oracle.cnn_conv(inp, W, b, bf16=True)
        mag = oracle.cnn_conv(np.abs(_bf16(inp)), np.abs(_bf16(W)), np.zeros(32))
        bound = np.sqrt(K) * U32 * mag + U32 * (np.abs(b)[None, :, None, None] + np.abs(ref)) + 1e-30
        _check(f"z{l}", acts[l], ref, bound)
        inp = _bf16(np.maximum(acts[l], 0.0))  # the GPU's own next-layer input
    # the head on the GPU's own last layer
    pooled = np.maximum(acts[2], 0.0).mean(axis=(2, 3))
    ref_logits = pooled @ _get(p, "Wh").T + _get(p, "bh")
    np.testing.assert_allclose(logits.cpu().numpy(), ref_logits, rtol=1e-5, atol=1e-5)


def test_backward_layer_by_layer_parity():
    """Every gradient entry against the oracle's adjoint of the same layer,
    fed the GPU's own operands: the layer input (BF16 of the GPU's previous
    activations), its pre-activation (ReLU mask) and the upstream gradient the
    GPU's backward consumed.  Weight gradients: K = B*256 pixel products of
    BF16 operands, |err| <= sqrt(K) 2^-24 sum |g a|; input gradients: K = 288
    products and a 9-term tap sum, sqrt(K) 2^-24 sum |g w|; bias gradients:
    FP32 sums of K = B*256 terms, sqrt(K) 2^-24 sum |g|.  The head (pooling,
    FP32 softmax with expf/logf, batch sums) is held to 2^-24 x 512 of the
    magnitude of its terms."""
    import torch
    t, p, x, xd = _setup(2, B=6)
    B = x.shape[0]
    labels = np.array([0, 1, 2, 2, 1, 0], np.int32)
    lab = torch.from_numpy(labels).cuda()
    g = torch.zeros(t.nparams, dtype=torch.float32, device="cuda")
    _, acts = t.forward(xd, acts=True)
    loss, dacts = t.loss_grad(xd, lab, g, dacts=True)
    torch.cuda.synchronize()
    z = _nhwc(acts, B)
    da = _nhwc(dacts, B)
    gg = g.cpu().numpy().astype(np.float64)
    sl = _slices()

    def grad_of(name):
        a, b, shape = sl[name]
        return gg[a:b].reshape(shape)

    # head: loss, Wh, bh and the upstream gradient of layer 3
    a3 = np.maximum(z[2], 0.0)
    oloss, _, gWh, gbh, da3 = oracle.cnn_head(p, a3, labels)
    # |d loss / d logit| <= 1/B per sample, so the terms of the head sums are
    # bounded by pooled / B (Wh), 1 / B (bh) and |Wh| / (256 B) (dA3)
    tol = 512 * U32
    pooled_sum = a3.mean(axis=(2, 3)).sum(axis=0) / B
    _check("loss", float(loss.item()), oloss, tol * (abs(oloss) + 1.0))
    _check("Wh", grad_of("Wh"), gWh, tol * (np.abs(gWh) + pooled_sum[None, :]))
    _check("bh", grad_of("bh"), gbh, tol * (np.abs(gbh) + 1.0))
    scale = np.abs(_get(p, "Wh")).sum(axis=0)[None, :, None, None] / (256.0 * B)
    _check("dA3", da[2], da3, tol * (np.abs(da3) + scale))
    # convolution layers, from the last to the first
    inputs = [x.astype(np.float64), np.maximum(z[0], 0.0), np.maximum(z[1], 0.0)]
    for l in (2, 1, 0):
        W = _get(p, f"W{l}")
        dz = np.where(z[l] > 0.0, da[l], 0.0)
        gW, gb, din = oracle.cnn_conv_backward(inputs[l], W, dz, bf16=True)
        mW, mb, mdin = oracle.cnn_conv_backward(np.abs(inputs[l]), np.abs(W), np.abs(dz), bf16=True)
        Kp = B * 256
        _check(f"W{l}", grad_of(f"W{l}"), gW, np.sqrt(Kp) * U32 * mW + 1e-30)
        _check(f"b{l}", grad_of(f"b{l}"), gb, np.sqrt(Kp) * U32 * mb + 1e-30)
        if l > 0:
            _check(f"dA{l}", da[l - 1], din, np.sqrt(288 + 9) * U32 * mdin + 1e-30)


def test_gradient_is_deterministic():
    """Fixed-order reductions: two evaluations give the same bits."""
    import torch
    t, p, x, xd = _setup(4, B=40)
    lab = torch.from_numpy(np.arange(40, dtype=np.int32) % 3).cuda()
    g1 = torch.zeros(t.nparams, dtype=torch.float32, device="cuda")
    g2 = torch.zeros_like(g1)
    l1 = t.loss_grad(xd, lab, g1)
    l2 = t.loss_grad(xd, lab, g2)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_training_learns_a_separable_task():
    """Adam on the GPU: three classes told apart by which input channel holds
    a bump; the loss falls and held-out accuracy exceeds 0.95."""
    import torch
    rng = np.random.default_rng(3)
    t = af.Tagger(NIN)
    p = (rng.standard_normal(t.nparams) * 0.1).astype(np.float32)
    t.set_params(p)

    def batch(n):
        lab = rng.integers(0, 3, n).astype(np.int32)
        x = rng.standard_normal((n, NIN, 16, 16)).astype(np.float32) * 0.5
        yy, xx = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
        for i in range(n):
            cy, cx = rng.integers(3, 13, 2)
            x[i, lab[i] * 4] += 3.0 * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / 6.0)
        return torch.from_numpy(x).cuda(), torch.from_numpy(lab).cuda()

    losses = []
    for it in range(150):
        xb, lb = batch(64)
        loss = t.loss_grad(xb, lb)
        t.adam_step(3e-3)
        if it % 10 == 0:
            losses.append(float(loss.item()))
    xt, lt = batch(256)
    pred = t.forward(xt).argmax(dim=1)
    acc = float((pred == lt.long()).float().mean().item())
    print(f"[gpu-cnn] training losses {losses[0]:.3f} -> {losses[-1]:.3f}, accuracy {acc:.3f}", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    assert acc > 0.95


def test_tag_fallback_rules():
    """Non-finite network output falls back to the plain tags; a network that
    always says refine makes every leaf below lmax refine; coarsening needs
    both to agree."""
    import torch
    m, n0, lmax = 16, 2, 2
    prob = af.Problem(eq=1, prec=af.FP32, m=m, n0x=n0, n0y=n0, lmax=lmax, c=1.0)
    ctx = af.Context(prob)
    leaves = afsynth.diagonal_leaves(n0, 1)
    blocks = []
    data = afsynth.gaussian_pulse(1)
    for (l, ix, iy) in leaves:
        dx = prob.dx(l)
        blocks.append(afsynth.dofs_block(data, m, 2, ix * m * dx, iy * m * dx, dx, dx, 4))
    h = af.Hierarchy(ctx, leaves)
    b0 = af.blocks_to_state(ctx, blocks)
    bufs = [b0, b0]
    t = af.Tagger(NIN)
    n = len(leaves)
    plain = torch.tensor([(-1, 0, 1)[k % 3] for k in range(n)], dtype=torch.int8, device="cuda")
    nan = np.full(t.nparams, np.nan, np.float32)
    t.set_params(nan)
    tags, learned = t.tag(ctx, h, bufs, 0, plain)
    torch.cuda.synchronize()
    pl = plain.cpu().numpy()
    lv = np.array([l for l, _, _ in leaves])
    want = np.where((pl == 1) & (lv >= lmax), 0, np.where((pl == -1) & (lv == 0), 0, pl))  # level limits
    np.testing.assert_array_equal(tags.cpu().numpy(), want)
    assert (learned.cpu().numpy() == 2).all()
    p = np.zeros(t.nparams, np.float32)
    a, b, _ = _slices()["bh"]
    p[a + 2] = 10.0  # refine logit dominates
    t.set_params(p)
    tags, learned = t.tag(ctx, h, bufs, 0, plain)
    torch.cuda.synchronize()
    tg = tags.cpu().numpy()
    for k, (l, _, _) in enumerate(leaves):
        assert tg[k] == (1 if l < lmax else 0)
    p[a + 2] = 0.0
    p[a + 0] = 10.0  # coarsen logit dominates: coarsen only where plain agrees
    t.set_params(p)
    tags, _ = t.tag(ctx, h, bufs, 0, plain)
    torch.cuda.synchronize()
    tg = tags.cpu().numpy()
    pl = plain.cpu().numpy()
    for k, (l, _, _) in enumerate(leaves):
        want = -1 if (pl[k] == -1 and l > 0) else (1 if (pl[k] == 1 and l < lmax) else 0)
        assert tg[k] == want, (k, l, pl[k], tg[k])


def test_features_layout():
    """Feature channel 4q+k is component q's DOF kind k at the owned position
    of each cell, channel 12 the level, after standardisation."""
    import torch
    m, n0 = 16, 2
    prob = af.Problem(eq=1, prec=af.FP64, m=m, n0x=n0, n0y=n0, lmax=1, c=1.0)
    ctx = af.Context(prob)
    leaves = afsynth.uniform_leaves(n0, n0, 1)
    rng = np.random.default_rng(9)
    blocks = [{k: rng.standard_normal((3, m + 5, m + 5)) for k in af.KINDS} for _ in leaves]
    h = af.Hierarchy(ctx, leaves)
    b0 = af.blocks_to_state(ctx, blocks)
    t = af.Tagger(NIN)
    mean = np.arange(NIN, dtype=np.float32) * 0.1
    inv = 1.0 + np.arange(NIN, dtype=np.float32) * 0.01
    t.set_normalization(mean, inv)
    x = t.features(ctx, h, [b0, b0], 0).cpu().numpy()
    for k, b in enumerate(blocks):
        for q in range(3):
            for kk, kind in enumerate(af.KINDS):
                ch = 4 * q + kk
                ref = (b[kind][q, 2:2 + m, 2:2 + m].astype(np.float32) - mean[ch]) * inv[ch]
                np.testing.assert_allclose(x[k, ch], ref, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(x[k, 12], (1.0 - mean[12]) * inv[12], rtol=1e-6)
