"""Several coarse steps in one call (af_amr_coarse_steps): the result must be
bit for bit that of the same number of af_amr_coarse_step calls (the last
fix of a step shares a launch with the next step's vertex copies), for
acoustics and advection, FP32 and FP64, subcycled and global stepping; the
flux registers are left zero either way."""
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


CASES = [
    # name, eq, m, n0, lmax, data, theta
    ("ac16", af.ACOUSTICS, 16, 4, 3, lambda: afsynth.wave_packet(5, alpha=200.0, kdiv=4), (24.0, 6.0)),
    ("adv16", af.ADVECTION, 16, 4, 2, lambda: afsynth.tanh_disc(), (4.0, 1.0)),
]


@pytest.mark.parametrize("global_step", [False, True], ids=["subcycled", "global"])
@pytest.mark.parametrize("prec", [af.FP32, af.FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_coarse_steps_equal_single_steps(case, prec, global_step):
    from paper_2205_07572_amd.amr import AMRRun, TagRule, initial_hierarchy
    name, eq, m, n0, lmax, data, theta = case
    data = data()
    kw = dict(c=1.0) if eq == af.ACOUSTICS else dict(a=1.0, b=0.5)
    prob = af.Problem(eq=eq, prec=prec, m=m, n0x=n0, n0y=n0, lmax=lmax, **kw)

    def block_fn(l, ix, iy):
        dx = prob.dx(l)
        return afsynth.dofs_block(data, m, 2, ix * m * dx, iy * m * dx, dx, dx, 4)

    run = initial_hierarchy(prob, block_fn, TagRule(af.TAG_GRADIENT, 0, *theta))
    leaves = run.hier.leaves()
    counts = np.bincount([l for l, _, _ in leaves], minlength=lmax + 1)
    assert counts[lmax] > 0, counts
    blocks = run.blocks()
    nsteps = 3
    dt0 = 0.4 * prob.dx(lmax if global_step else 0)
    out = []
    for multi in (False, True):
        r = AMRRun(prob, leaves, lambda l, ix, iy: blocks[leaves.index((l, ix, iy))])
        if multi:
            r.mask = r.ctx.amr_coarse_steps(r.hier, r.bufs, r.mask, dt0, nsteps, r.reg, global_step=global_step)
        else:
            for _ in range(nsteps):
                r.mask = r.ctx.amr_coarse_step(r.hier, r.bufs, r.mask, dt0, r.reg, global_step=global_step)
        out.append((r.mask, r.blocks(), float(r.reg.abs().max())))
        del r
    print(f"[coarse-steps] {name} prec={prec} global={global_step}: {len(leaves)} leaves per level "
          f"{counts.tolist()}", flush=True)
    (mask_s, bs, reg_s), (mask_m, bm, reg_m) = out
    assert mask_s == mask_m, (mask_s, mask_m)
    assert reg_s == 0.0 and reg_m == 0.0, (reg_s, reg_m)
    cm = closed_masks(m)
    for k, (a, b) in enumerate(zip(bs, bm)):
        for kind in af.KINDS:
            x, y = a[kind][:, cm[kind]], b[kind][:, cm[kind]]
            assert np.array_equal(x, y), (name, k, leaves[k], kind, np.abs(x - y).max())
