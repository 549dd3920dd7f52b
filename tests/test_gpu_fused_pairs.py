"""Fused pairs of finest-level substeps in the batched coarse step: the same
hierarchy stepped with the option on and off must give bit-identical leaf
data (interiors and closed-square nodes) and the same level-buffer mask, for
acoustics and advection, FP32 and FP64, m = 16 and m = 8, eager and graph
replay.  Parity of the fused path with the oracle is covered by the
adaptive tests, which run with the option's default (on)."""
import os

import numpy as np
import pytest

import afsynth
import paper_2205_07572_amd as af
from harness import closed_masks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU on this machine")
    assert torch.cuda.is_available(), "GPU present but torch.cuda.is_available() is False"


def build(eq, prec, m, n0, lmax, data, theta):
    """A hierarchy with levels 0..lmax from gradient tags of the data (on
    component 0), as the adaptive runs build it."""
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    kw = dict(c=1.0) if eq == af.ACOUSTICS else dict(a=1.0, b=0.5)
    prob = af.Problem(eq=eq, prec=prec, m=m, n0x=n0, n0y=n0, lmax=lmax, **kw)

    def block_fn(l, ix, iy):
        dx = prob.dx(l)
        return afsynth.dofs_block(data, m, 2, ix * m * dx, iy * m * dx, dx, dx, 4)

    return initial_hierarchy(prob, block_fn, TagRule(af.TAG_GRADIENT, 0, *theta)), block_fn


def twin_runs(eq, prec, m, n0, lmax, data, theta, steps, use_graph):
    from paper_2205_07572_amd.amr import AMRRun
    run, block_fn = build(eq, prec, m, n0, lmax, data, theta)
    leaves = run.hier.leaves()
    counts = np.bincount([l for l, _, _ in leaves], minlength=lmax + 1)
    assert counts[lmax] > 0, counts
    blocks = run.blocks()
    out = []
    for fused in (True, False):
        r = AMRRun(run.prob, leaves, lambda l, ix, iy: blocks[leaves.index((l, ix, iy))])
        r.ctx.fused_pairs = fused
        assert r.ctx.fused_pairs == fused
        dt0 = 0.4 * r.prob.dx(0)
        r.coarse_steps(dt0, steps, use_graph=use_graph)
        out.append((r.mask, r.blocks()))
        del r
    return leaves, counts, out


CASES = [
    # eq, prec, m, n0, lmax, data, theta
    ("ac16", af.ACOUSTICS, 16, 4, 3, lambda: afsynth.wave_packet(5, alpha=200.0, kdiv=4), (24.0, 6.0)),
    ("ac8", af.ACOUSTICS, 8, 6, 2, lambda: afsynth.gaussian_pulse(3), (6.0, 1.5)),
    ("adv16", af.ADVECTION, 16, 4, 2, lambda: afsynth.tanh_disc(), (4.0, 1.0)),
]


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("prec", [af.FP32, af.FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_pairs_bit_identical(case, prec, use_graph):
    name, eq, m, n0, lmax, data, theta = case
    leaves, counts, ((mask_f, bf), (mask_u, bu)) = twin_runs(eq, prec, m, n0, lmax, data(), theta, 3, use_graph)
    print(f"[fused-pairs] {name} prec={prec} graph={use_graph}: {len(leaves)} leaves per level {counts.tolist()}",
          flush=True)
    assert mask_f == mask_u, (mask_f, mask_u)
    cm = closed_masks(m)
    for k, (a, b) in enumerate(zip(bf, bu)):
        for kind in af.KINDS:
            x, y = a[kind][:, cm[kind]], b[kind][:, cm[kind]]
            assert np.array_equal(x, y), (name, k, leaves[k], kind, np.abs(x - y).max())


def test_fused_pairs_option():
    prob = af.Problem(eq=af.ACOUSTICS, prec=af.FP32, m=16, n0x=2, n0y=2, lmax=2, c=1.0)
    ctx = af.Context(prob)
    assert ctx.fused_pairs
    ctx.fused_pairs = False
    assert not ctx.fused_pairs
    ctx.fused_pairs = True
    assert ctx.fused_pairs
