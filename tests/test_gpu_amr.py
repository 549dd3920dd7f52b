"""GPU adaptive runs (Sec. 3) against the oracle: initial hierarchy from the
tagger, coarse steps with subcycling and the conservative fix, regrids with
tags replayed from the oracle (FP64 1e-12 relative L-infinity), and global
conservation across regrids."""
import os

import numpy as np
import pytest

import afsynth
import oracle
import paper_2205_07572_amd as af
from harness import KINDS, closed_masks, oracle_blocks, rel_linf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU on this machine")
    assert torch.cuda.is_available(), "GPU present but torch.cuda.is_available() is False"


def _block_fn(prob, data):
    def fn(l, ix, iy):
        dx, dy = prob.dx(l), prob.dy(l)
        return afsynth.dofs_block(data, prob.m, 2, prob.x0 + ix * prob.m * dx, prob.y0 + iy * prob.m * dy, dx, dy, 4)
    return fn


@pytest.mark.parametrize("eq", [1, 0])
def test_adaptive_run_matches_oracle_with_tag_replay(eq):
    """Config-3-like acoustics (Gaussian pulse, gradient tags) and advection
    (max-min tags): 3 cycles of (regrid, 2 coarse steps)."""
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    m, n0, lmax = 8, 4, 2
    if eq == 1:
        prob = af.Problem(eq=1, prec=af.FP64, m=m, n0x=n0, n0y=n0, lmax=lmax, c=1.0)
        data = afsynth.gaussian_pulse(11, alpha=60.0)
        rule = TagRule(af.TAG_GRADIENT, 0, 2.0, 0.5)
    else:
        prob = af.Problem(eq=0, prec=af.FP64, m=m, n0x=n0, n0y=n0, lmax=lmax, a=1.0, b=0.5)
        data = afsynth.fourier_modes(11, nmodes=3, kmax=2)
        rule = TagRule(af.TAG_MAXMIN, 0, 1.2, 0.4)
    run = initial_hierarchy(prob, _block_fn(prob, data), rule)
    leaves = run.hier.leaves()
    assert len(set(l for l, _, _ in leaves)) >= 2, leaves
    o = oracle.Hier(eq, m, n0, n0, lmax, a=prob.a, b=prob.b, c=prob.c)
    o.set_leaves(leaves)
    for k, b in enumerate(run.blocks()):
        o.set_block(k, b)
    dt0 = 0.4 * prob.dx(0)
    s0 = run.total()
    for cycle in range(3):
        run.coarse_steps(dt0, 2)
        o.run(dt0, 2)
        err = rel_linf(run.blocks(), oracle_blocks(o), closed_masks(m))
        assert err.max() <= 1e-12, (cycle, err)
        o.fill()
        otags, ovals = o.tag(rule.mode, rule.comp, rule.theta_r, rule.theta_c)
        gtags, gvals = run.tags(rule)
        np.testing.assert_allclose(gvals, ovals, rtol=1e-10, atol=1e-12)
        run.regrid(tags=otags)
        o.regrid(otags)
        assert run.hier.leaves() == o.leaves()
    err = rel_linf(run.blocks(), oracle_blocks(o), closed_masks(m))
    assert err.max() <= 1e-12, err
    s1 = run.total()
    scale = sum(np.abs(b["avg"][:, 2:2 + m, 2:2 + m]).sum() * prob.dx(l) * prob.dy(l)
                for b, (l, _, _) in zip(run.blocks(), run.hier.leaves()))
    assert np.abs(s1 - s0).max() <= 1e-13 * scale, (s0, s1)
    assert run.stats.regrids == 3


def test_adaptive_run_fp32_conservation():
    """FP32 bulk, FP64 registers and sums: conservation across regrids to
    FP32 round-off (bound 1e-6 of the sum of |Q| x area)."""
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    m, n0, lmax = 16, 4, 2
    prob = af.Problem(eq=1, prec=af.FP32, m=m, n0x=n0, n0y=n0, lmax=lmax, c=1.0)
    data = afsynth.gaussian_pulse(5, alpha=120.0)
    rule = TagRule(af.TAG_GRADIENT, 0, 2.0, 0.5)
    run = initial_hierarchy(prob, _block_fn(prob, data), rule)
    s0 = run.total()
    dt0 = 0.4 * prob.dx(0)
    for _ in range(4):
        run.coarse_steps(dt0, 4)
        run.regrid(rule)
    s1 = run.total()
    scale = sum(np.abs(b["avg"][:, 2:2 + m, 2:2 + m]).sum() * prob.dx(l) * prob.dy(l)
                for b, (l, _, _) in zip(run.blocks(), run.hier.leaves()))
    drift = np.abs(s1 - s0).max() / scale
    print(f"[gpu-amr] fp32 conservation drift {drift:.3e} over 16 coarse steps and 4 regrids, "
          f"leaves {run.stats.leaves_history}", flush=True)
    assert drift < 1e-6
