"""af_reduce_sum_noalloc (the allocation-free conservation sum) against
af_reduce_sum through the C ABI: same sums, bit for bit, on two calls in a
row, the second on a smaller hierarchy (the static scratch keeps the first
call's partial sums; every entry the second call reads is rewritten)."""
import os

import numpy as np
import pytest

import afsynth
import paper_2205_07572_amd as af
from harness import leaf_blocks, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU on this machine")
    assert torch.cuda.is_available(), "GPU present but torch.cuda.is_available() is False"


def _case(prec, n0, lmax, leaves, seed):
    import torch
    prob = make_problem(1, prec, 8, n0=n0, lmax=lmax, c=1.0)
    ctx = af.Context(prob)
    h = af.Hierarchy(ctx, leaves)
    blocks = leaf_blocks(prob, leaves, afsynth.gaussian_pulse(seed))
    b0 = af.blocks_to_state(ctx, blocks)
    b1 = torch.roll(b0, 1, dims=-1).contiguous()  # a different second buffer, so the mask matters
    h.leaf_xy_ptr()  # uploads the hierarchy's device tables (the no-alloc call does not)
    return ctx, h, [b0, b1]


@pytest.mark.parametrize("prec", [af.FP64, af.FP32])
def test_noalloc_sum_matches_reduce_sum_twice(prec):
    import torch
    print(f"[no-alloc] reduce_sum_noalloc prec={prec}", flush=True)
    big = _case(prec, 4, 2, afsynth.diagonal_leaves(4, 1), 3)
    small = _case(prec, 2, 1, afsynth.diagonal_leaves(2, 0), 4)
    assert len(small[1]) < len(big[1])
    for (ctx, h, bufs), mask in ((big, 0b010), (small, 0b01)):
        ref = torch.zeros(3, dtype=torch.float64, device="cuda")
        got = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.reduce_sum(h, bufs, mask, ref)
        ctx.reduce_sum_noalloc(h, bufs, mask, got)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(r).all() and np.any(r != 0.0)
        np.testing.assert_array_equal(g, r)
