"""GPU parity for solid-body rotation (Sec. 4.2, a = -omega y, b = omega x on
[-1, 1]^2): the patch step against the oracle's, subcycled coarse steps
against the oracle's recursion, constant states, and the paper's Table 2
error as a soft pin."""
import os

import numpy as np
import pytest

import afsynth
import oracle
import paper_2205_07572_amd as af
from harness import KINDS, closed_masks, rel_linf

pytestmark = pytest.mark.gpu

OMEGA = np.pi
FP64_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU on this machine")
    assert torch.cuda.is_available(), "GPU present but torch.cuda.is_available() is False"


def _problem(prec, m, n0, lmax=0):
    return af.Problem(eq=af.ROTATION, prec=prec, m=m, n0x=n0, n0y=n0, lmax=lmax, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0,
                      omega=OMEGA)


def _rand_blocks(rng, n, m):
    from harness import valid_masks
    vm = valid_masks(m)
    out = []
    for _ in range(n):
        b = {}
        for k in KINDS:
            a = rng.standard_normal((1, m + 5, m + 5))
            a[:, ~vm[k]] = 0.0
            b[k] = a
        out.append(b)
    return out


@pytest.mark.parametrize("m", [8, 16, 32])
@pytest.mark.parametrize("region", [0, 1])
def test_rotation_patch_step_parity_fp64(m, region):
    """Patches at several places of the domain (positions through leaf_xy),
    every tile height, flux registers on all sides."""
    import torch
    print(f"[gpu-rotation] patch_step m={m} region={region}", flush=True)
    rng = np.random.default_rng(7 * m + region)
    n0 = 4
    prob = _problem(af.FP64, m, n0)
    ctx = af.Context(prob)
    pos = [(0, 0), (3, 1), (1, 2), (2, 3)]
    blocks = _rand_blocks(rng, len(pos), m)
    xy = torch.tensor(pos, dtype=torch.int32, device="cuda")
    dx = prob.dx(0)
    dt = 0.9 * dx / OMEGA  # largest speed in either direction is omega * 1
    for ty in {8: [8], 16: [8, 16], 32: [4, 8]}[m]:
        ctx.tile = ty
        tin = af.blocks_to_state(ctx, blocks)
        tout = torch.zeros_like(tin)
        reg = torch.zeros((len(pos), 4, m, 1), dtype=torch.float64, device="cuda")
        mask = torch.full((len(pos),), 15, dtype=torch.uint8, device="cuda")
        ctx.patch_step(tin, tout, 0, len(pos), 0, dt, region, reg, mask, leaf_xy=xy)
        torch.cuda.synchronize()
        got = af.state_to_blocks(ctx, tout)
        regs = reg.cpu().numpy()
        mk = closed_masks(m, region)
        for p, (ix, iy) in enumerate(pos):
            flux4 = np.zeros((4, m, 1))
            ref = oracle.patch_step_rot(m, blocks[p], -1.0 + ix * m * dx, -1.0 + iy * m * dx, dx, dx, dt, OMEGA,
                                        region=region, flux4=flux4, side_mask=15)
            err = rel_linf([got[p]], [ref], mk)
            assert err.max() <= FP64_TOL, (ty, p, err)
            np.testing.assert_allclose(regs[p], flux4, rtol=1e-12, atol=1e-14 * np.abs(flux4).max())


def test_rotation_needs_leaf_positions():
    import torch
    prob = _problem(af.FP64, 8, 2)
    ctx = af.Context(prob)
    t = ctx.new_state(1)
    with pytest.raises(af.AFError) as e:
        ctx.patch_step(t, torch.zeros_like(t), 0, 1, 0, 0.01, 0)
    assert e.value.status == af._lib.AF_ERR_ARG
    with pytest.raises(af.AFError) as e:  # CFL with the largest speed omega * 1
        ctx.patch_step(t, torch.zeros_like(t), 0, 1, 0, 1.01 * prob.dx(0) / OMEGA, 0,
                       leaf_xy=torch.zeros((1, 2), dtype=torch.int32, device="cuda"))
    assert e.value.status == af._lib.AF_ERR_CFL


def _amr(prec, leaves, n0, lmax, m, nsteps, data, use_graph=False):
    import torch
    prob = _problem(prec, m, n0, lmax)
    ctx = af.Context(prob)
    h = af.Hierarchy(ctx, leaves)
    blocks = []
    for (l, ix, iy) in leaves:
        dx = prob.dx(l)
        blocks.append(afsynth.dofs_block(data, m, 2, -1.0 + ix * m * dx, -1.0 + iy * m * dx, dx, dx, 6))
    b0 = af.blocks_to_state(ctx, blocks)
    bufs = [b0, torch.zeros_like(b0)]
    reg = torch.zeros((len(leaves), 4, m, 1), dtype=torch.float64, device="cuda")
    s_in = torch.zeros(1, dtype=torch.float64, device="cuda")
    s_out = torch.zeros_like(s_in)
    mask = 0
    ctx.ghost_fill(h, bufs, mask, 0, 0)
    ctx.reduce_sum(h, bufs, mask, s_in)
    dt0 = 0.6 * prob.dx(0) / OMEGA
    for _ in range(nsteps):
        mask = ctx.amr_coarse_step(h, bufs, mask, dt0, reg, use_graph=use_graph)
    ctx.reduce_sum(h, bufs, mask, s_out)
    torch.cuda.synchronize()
    g0, g1 = af.state_to_blocks(ctx, bufs[0]), af.state_to_blocks(ctx, bufs[1])
    got = [g1[k] if (mask >> leaves[k][0]) & 1 else g0[k] for k in range(len(leaves))]
    return got, blocks, float(s_in.item()), float(s_out.item()), dt0, prob


def _layouts():
    three = [(0, ix, iy) for iy in range(4) for ix in range(4) if not (1 <= ix <= 2 and 1 <= iy <= 2)]
    three += [(1, ix, iy) for iy in range(2, 6) for ix in range(2, 6) if not (3 <= ix <= 4 and 3 <= iy <= 4)]
    three += [(2, ix, iy) for iy in range(6, 10) for ix in range(6, 10)]
    return {"diagonal": (4, 1, afsynth.diagonal_leaves(4, 0)), "three": (4, 2, afsynth.sort_leaves(three))}


@pytest.mark.parametrize("layout", ["diagonal", "three"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_rotation_amr_parity_fp64(layout, use_graph):
    """Subcycled coarse steps with the conservative fix against the oracle,
    and global conservation (data negligible on the boundary)."""
    n0, lmax, leaves = _layouts()[layout]
    print(f"[gpu-rotation] amr {layout} graph={use_graph}", flush=True)
    m, nsteps = 8, 3
    data = afsynth.solid_body(afsynth.gauss_q0(0.15, 0.1, 60.0), OMEGA)
    got, blocks, s_in, s_out, dt0, prob = _amr(af.FP64, leaves, n0, lmax, m, nsteps, data, use_graph)
    h = oracle.Hier(2, m, n0, n0, lmax, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, omega=OMEGA)
    h.set_leaves(leaves)
    for k, b in enumerate(blocks):
        h.set_block(k, b)
    h.fill(0, 0)
    h.run(dt0, nsteps)
    ref = [h.get_block(k) for k in range(len(leaves))]
    err = rel_linf(got, ref, closed_masks(m, 0))
    assert err.max() <= FP64_TOL, err
    assert abs(s_out - s_in) <= 1e-13 * abs(s_in)


def test_rotation_constant_state_amr():
    """The Remark of Sec. 4.2 on the GPU, with subcycling: a constant stays
    constant to round-off."""
    n0, lmax, leaves = _layouts()["three"]
    got, _, _, _, _, _ = _amr(af.FP64, leaves, n0, lmax, 8, 6, afsynth.polynomial([{(0, 0): 0.7}]))
    for b in got:
        assert np.abs(b["avg"][0, 2:10, 2:10] - 0.7).max() <= 1e-13


def test_rotation_fp32_error_bound():
    """FP32 bulk against the FP64 oracle on a smooth field over 3 coarse
    steps: relative L-infinity below 1e-5."""
    n0, lmax, leaves = _layouts()["diagonal"]
    m = 16
    data = afsynth.solid_body(afsynth.gauss_q0(0.15, 0.1, 60.0), OMEGA)
    got, blocks, _, _, dt0, _ = _amr(af.FP32, leaves, n0, lmax, m, 3, data)
    h = oracle.Hier(2, m, n0, n0, lmax, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, omega=OMEGA)
    h.set_leaves(leaves)
    for k, b in enumerate(blocks):
        h.set_block(k, {kk: v.astype(np.float32).astype(np.float64) for kk, v in b.items()})
    h.fill(0, 0)
    h.run(dt0, 3)
    ref = [h.get_block(k) for k in range(len(leaves))]
    err = rel_linf(got, ref, closed_masks(m, 0))
    print(f"[gpu-rotation] fp32 rel L-inf {err.max():.2e}", flush=True)
    assert err.max() <= 1e-5, err


def _disc_run(level, T=1.0, cfl=0.6, m=32, speed=OMEGA):
    """Uniform grid of level `level` (16 * 2^level cells per side) on
    [-1, 1]^2, the smoothed disc of eq. AdvH rotated to time T at the given
    Courant number relative to `speed` (default omega * 1, the largest speed
    along either axis); returns the L1 error of the averages, area-weighted
    and divided by the domain area."""
    import math
    import torch
    N = 16 << level
    n0 = N // m
    data = afsynth.solid_body(afsynth.disc_q0(0.15, 0.02, 0.5, 0.5), OMEGA)
    prob = _problem(af.FP64, m, n0)
    ctx = af.Context(prob)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    h = af.Hierarchy(ctx, leaves)
    d0 = afsynth.dofs_periodic(data, N, N, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, nq=4)
    blk = afsynth.periodic_to_blocks(d0, m)
    b0 = af.blocks_to_state(ctx, [{k: blk[k][p] for k in KINDS} for p in range(n0 * n0)])
    bufs = [b0, torch.zeros_like(b0)]
    reg = torch.zeros((len(leaves), 4, m, 1), dtype=torch.float64, device="cuda")
    dx = 2.0 / N
    n = math.ceil(T / (cfl * dx / speed))
    mask = 0
    for _ in range(n):
        mask = ctx.amr_coarse_step(h, bufs, mask, T / n, reg)
    got = af.state_to_blocks(ctx, bufs[mask & 1])
    avg = np.zeros((N, N))
    for p, (_, ix, iy) in enumerate(leaves):
        avg[iy * m:(iy + 1) * m, ix * m:(ix + 1) * m] = got[p]["avg"][0, 2:2 + m, 2:2 + m]
    ex = afsynth.dofs_periodic(afsynth.InitialData(1, lambda x, y: data.exact(x, y, T)), N, N, x0=-1.0, y0=-1.0,
                               lx=2.0, ly=2.0, nq=4)["avg"][0]
    return float(np.abs(avg - ex).sum() * dx * dx / 4.0)


def test_rotation_table2_soft_pin():
    """Table 2 (left, uniform levels 6 and 7): L1 errors 4.599185e-06 and
    5.826258e-07, EOC 2.9807, after a half rotation.  The paper does not state
    the speed its CFL 0.6 refers to.  With the largest axis speed (pi) the
    errors are 1.26x the printed ones at both levels, with the speed at the
    disc's orbit (pi / sqrt 2) 0.92x: the printed errors lie between the two
    readings, each ratio is pinned to 5%, it is the same at both levels, and
    the EOC agrees to 0.02."""
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", "table2_rotation.json")) as f:
        paper = json.load(f)["uniform"]
    e6, e7 = _disc_run(6), _disc_run(7)
    eoc = np.log2(e6 / e7)
    print(f"[gpu-rotation] table 2: level 6 {e6:.6e}, level 7 {e7:.6e}, EOC {eoc:.4f}", flush=True)
    r6, r7 = e6 / paper["6"], e7 / paper["7"]
    assert 1.20 <= r6 <= 1.32 and 1.20 <= r7 <= 1.32, (r6, r7)
    assert abs(r6 - r7) <= 0.02, (r6, r7)
    assert abs(eoc - paper["eoc_6_7"]) <= 0.02
    o6 = _disc_run(6, speed=OMEGA / np.sqrt(2.0)) / paper["6"]
    print(f"[gpu-rotation] table 2 with the orbit speed: level 6 ratio {o6:.4f}", flush=True)
    assert 0.87 <= o6 <= 0.97, o6


def test_rotation_adaptive_run_with_tag_replay():
    """Adaptive rotation run (max - min tags, the criterion of Sec. 4.1):
    three cycles of (2 coarse steps, regrid) against the oracle with the
    oracle's tags replayed; the position-dependent field follows the leaves
    through every change of layout."""
    from harness import oracle_blocks
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    print("[gpu-rotation] adaptive run", flush=True)
    m, n0, lmax = 8, 4, 2
    prob = _problem(af.FP64, m, n0, lmax)
    data = afsynth.solid_body(afsynth.gauss_q0(0.3, 0.1, 30.0), OMEGA)

    def block_fn(l, ix, iy):
        dx = prob.dx(l)
        return afsynth.dofs_block(data, m, 2, -1.0 + ix * m * dx, -1.0 + iy * m * dx, dx, dx, 4)

    rule = TagRule(af.TAG_MAXMIN, 0, 0.05, 0.01)
    run = initial_hierarchy(prob, block_fn, rule)
    o = oracle.Hier(2, m, n0, n0, lmax, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, omega=OMEGA)
    o.set_leaves(run.hier.leaves())
    for k, b in enumerate(run.blocks()):
        o.set_block(k, b)
    dt0 = 0.6 * prob.dx(0) / OMEGA
    changed = 0
    for cycle in range(3):
        run.coarse_steps(dt0, 2)
        o.run(dt0, 2)
        err = rel_linf(run.blocks(), oracle_blocks(o), closed_masks(m))
        assert err.max() <= FP64_TOL, (cycle, err)
        o.fill()
        otags, _ = o.tag(rule.mode, rule.comp, rule.theta_r, rule.theta_c)
        before = run.hier.leaves()
        run.regrid(tags=otags)
        o.regrid(otags)
        assert run.hier.leaves() == o.leaves()
        changed += run.hier.leaves() != before
    err = rel_linf(run.blocks(), oracle_blocks(o), closed_masks(m))
    assert err.max() <= FP64_TOL, err
    assert changed >= 2


def test_rotation_full_size_level6():
    """The timed configuration at full size: uniform level 6 (1024^2 as
    32^2 patches) on [-1, 1]^2, general path, two steps at Courant number 0.6
    against the oracle's periodic 1024^2 grid, every DOF compared."""
    import math
    import torch
    print("[gpu-rotation] full size level 6", flush=True)
    m, N = 32, 1024
    n0 = N // m
    data = afsynth.solid_body(afsynth.disc_q0(0.15, 0.02, 0.5, 0.5), OMEGA)
    prob = _problem(af.FP64, m, n0)
    ctx = af.Context(prob)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    h = af.Hierarchy(ctx, leaves)
    d0 = afsynth.dofs_periodic(data, N, N, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, nq=4)
    blk = afsynth.periodic_to_blocks(d0, m)
    b0 = af.blocks_to_state(ctx, [{k: blk[k][p] for k in KINDS} for p in range(n0 * n0)])
    bufs = [b0, torch.zeros_like(b0)]
    reg = torch.zeros((len(leaves), 4, m, 1), dtype=torch.float64, device="cuda")
    dt = 1.0 / math.ceil(1.0 / (0.6 * (2.0 / N) / OMEGA))
    mask = 0
    for _ in range(2):
        mask = ctx.amr_coarse_step(h, bufs, mask, dt, reg)
    got = af.state_to_blocks(ctx, bufs[mask & 1])
    from harness import periodic_interior
    g = periodic_interior(got, leaves, m, n0)
    ref = oracle.run_periodic_rot(d0, dt, 2, OMEGA, x0=-1.0, y0=-1.0)
    err = max(np.abs(g[k][0] - ref[k][0]).max() for k in KINDS) / np.abs(ref["avg"][0]).max()
    print(f"[gpu-rotation] full size rel L-inf {err:.2e}", flush=True)
    assert err <= FP64_TOL
