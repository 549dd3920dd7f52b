"""GPU parity: every entry point of libaf.so against the CPU oracle on the
same seeded inputs.  FP64 must match to 1e-12 relative L-infinity
(max |gpu - oracle| / max |oracle| per component, over averages and point
values); FP32 results are checked against stated bounds."""
import numpy as np
import pytest

import afsynth
import oracle
import paper_2205_07572_amd as af
from harness import (KINDS, closed_masks, leaf_blocks, make_problem, oracle_blocks, periodic_interior, rel_linf,
                     valid_masks)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import os
    torch = pytest.importorskip("torch")
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU on this machine")
    # on a GPU machine a GPU that torch cannot see is an error, not a skip
    assert torch.cuda.is_available(), "GPU present but torch.cuda.is_available() is False"
    print("[gpu-parity] device:", torch.cuda.get_device_name(0), flush=True)


def _torch():
    import torch
    return torch


def _rand_blocks(rng, n, ncomp, m):
    S1 = m + 5
    vm = valid_masks(m)
    out = []
    for _ in range(n):
        b = {}
        for k in KINDS:
            a = rng.standard_normal((ncomp, S1, S1))
            a[:, ~vm[k]] = 0.0
            b[k] = a
        out.append(b)
    return out


PHYS = {0: dict(a=0.8, b=-0.45), 1: dict(c=1.3)}


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("m", [8, 16, 32])
@pytest.mark.parametrize("region", [0, 1])
def test_patch_step_parity_fp64(eq, m, region):
    torch = _torch()
    print(f"[gpu-parity] patch_step eq={eq} m={m} region={region}", flush=True)
    rng = np.random.default_rng(100 * eq + m + region)
    prob = make_problem(eq, af.FP64, m, **PHYS[eq])
    ctx = af.Context(prob)
    nc = prob.ncomp
    blocks = _rand_blocks(rng, 3, nc, m)
    dx, dy = prob.dx(0), prob.dy(0)
    dt = (0.9 * min(dx / abs(prob.a), dy / abs(prob.b))) if eq == 0 else 0.45 * dx / prob.c
    for ty in {8: [8], 16: [8, 16], 32: [4, 8]}[m]:
        ctx.tile = ty
        tin = af.blocks_to_state(ctx, blocks)
        tout = torch.zeros_like(tin)
        reg = torch.zeros((3, 4, m, nc), dtype=torch.float64, device="cuda")
        mask = torch.tensor([15, 15, 15], dtype=torch.uint8, device="cuda")
        ctx.patch_step(tin, tout, 1, 2, 0, dt, region, reg, mask)
        torch.cuda.synchronize()
        got = af.state_to_blocks(ctx, tout)
        regs = reg.cpu().numpy()
        mk = closed_masks(m, region)
        assert all(np.all(got[0][k] == 0) for k in KINDS)  # patch 0 untouched
        for p in (1, 2):
            flux4 = np.zeros((4, m, nc))
            ref = oracle.patch_step(eq, m, blocks[p], dx, dy, dt, region=region, a=prob.a, b=prob.b, c=prob.c,
                                    flux4=flux4, side_mask=15)
            err = rel_linf([got[p]], [ref], mk)
            assert err.max() <= FP64_TOL, (ty, p, err)
            np.testing.assert_allclose(regs[p], flux4, rtol=1e-12, atol=1e-14 * np.abs(flux4).max())


@pytest.mark.parametrize("eq", [0, 1])
def test_patch_step_fp32_error_bound(eq):
    """FP32 step against the FP64 oracle on O(1) random data: relative
    L-infinity below 2e-6 (a few ulps of FP32 over ~100-term stencils)."""
    torch = _torch()
    rng = np.random.default_rng(7 + eq)
    m = 16
    prob = make_problem(eq, af.FP32, m, **PHYS[eq])
    ctx = af.Context(prob)
    blocks = _rand_blocks(rng, 1, prob.ncomp, m)
    dx = prob.dx(0)
    dt = 0.9 * dx / 0.8 if eq == 0 else 0.45 * dx / prob.c
    # the FP32 path starts from FP32-rounded data
    blocks32 = [{k: v.astype(np.float32).astype(np.float64) for k, v in b.items()} for b in blocks]
    tin = af.blocks_to_state(ctx, blocks32)
    tout = torch.zeros_like(tin)
    ctx.patch_step(tin, tout, 0, 1, 0, dt, 0)
    torch.cuda.synchronize()
    got = af.state_to_blocks(ctx, tout)
    ref = oracle.patch_step(eq, m, blocks32[0], dx, dx, dt, region=0, a=prob.a, b=prob.b, c=prob.c)
    err = rel_linf(got, [ref], closed_masks(m))
    print(f"[gpu-parity] fp32 patch step eq={eq} rel Linf={err}", flush=True)
    assert err.max() < 2e-6


def _uniform_run_gpu(ctx, prob, leaves, blocks, dt, nsteps, mode):
    """mode 'manual': fill + step per step via the public calls; 'driver':
    af_amr_coarse_step eager; 'graph': af_amr_coarse_step with hipGraph."""
    torch = _torch()
    h = af.Hierarchy(ctx, leaves)
    b0 = af.blocks_to_state(ctx, blocks)
    b1 = torch.zeros_like(b0)
    bufs = [b0, b1]
    mask = 0
    reg = torch.zeros((len(leaves), 4, prob.m, prob.ncomp), dtype=torch.float64, device="cuda")
    for _ in range(nsteps):
        if mode == "manual":
            ctx.ghost_fill(h, bufs, mask, 0, 0)
            cur = mask & 1
            ctx.patch_step(bufs[cur], bufs[cur ^ 1], 0, len(leaves), 0, dt, 0)
            mask ^= 1
        else:
            mask = ctx.amr_coarse_step(h, bufs, mask, dt, reg, use_graph=(mode == "graph"))
    torch.cuda.synchronize()
    return af.state_to_blocks(ctx, bufs[mask & 1]), h


@pytest.mark.parametrize("eq,n0,m,nsteps", [(0, 4, 16, 40), (1, 2, 16, 10)])
@pytest.mark.parametrize("mode", ["manual", "driver", "graph"])
def test_periodic_patches_match_single_grid(eq, n0, m, nsteps, mode):
    """Patches with same-level periodic ghost fill reproduce the oracle's
    single periodic grid (Sec. 3.1)."""
    print(f"[gpu-parity] periodic eq={eq} n0={n0} m={m} mode={mode}", flush=True)
    prob = make_problem(eq, af.FP64, m, n0=n0, **PHYS[eq])
    ctx = af.Context(prob)
    data = afsynth.fourier_modes(3) if eq == 0 else afsynth.gaussian_pulse(3)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    blocks = leaf_blocks(prob, leaves, data)
    N = n0 * m
    dt = 0.6 / N if eq == 0 else 0.4 / (N * prob.c)
    got, _ = _uniform_run_gpu(ctx, prob, leaves, blocks, dt, nsteps, mode)
    d0 = afsynth.dofs_periodic(data, N, N, nq=6)
    ref = oracle.run_periodic(eq, d0, dt, nsteps, a=prob.a, b=prob.b, c=prob.c)
    g = periodic_interior(got, leaves, m, n0)
    for q in range(prob.ncomp):
        den = max(np.abs(ref[k][q]).max() for k in KINDS)
        err = max(np.abs(g[k][q] - ref[k][q]).max() for k in KINDS) / den
        assert err <= FP64_TOL, (q, err)


# advection velocity patterns of the level advance: (a, b, Courant number of
# the faster direction).  "mixed" has both source-cell offsets at run time,
# "upwind" (a, b > 0, both directional Courant numbers below 1/2) takes the
# compile-time upwind variant, "steep" (transverse Courant number 0.8) makes
# the two time levels of the x-edges read different source cells.
VELOCITY = {"mixed": (0.8, -0.45, 0.4), "upwind": (1.0, 0.5, 0.4), "steep": (0.3, -1.0, 0.8)}


def _shape_cases():
    cases = []
    for eq, prec, m in [(0, af.FP32, 32), (0, af.FP64, 32), (0, af.FP32, 16), (0, af.FP64, 16),
                        (1, af.FP32, 16), (1, af.FP64, 16), (1, af.FP32, 32)]:
        ctx = af.Context(make_problem(eq, prec, m, n0=4))
        up_only = set(ctx.advance_shapes_upwind())
        for k, nt in ctx.advance_shapes():
            # the upwind-only shapes run only with the upwind velocity (other
            # weights fall back to the default shape: test_upwind_shape_fallback)
            vels = ["-"] if eq != 0 else (["upwind"] if (k, nt) in up_only else list(VELOCITY))
            for vel in vels:
                cases.append((eq, prec, m, k, nt, vel))
    return cases


@pytest.mark.parametrize("prec", [af.FP32, af.FP64], ids=["fp32", "fp64"])
def test_upwind_shape_fallback(prec):
    """An upwind-only shape with weights of another pattern: af_level_advance
    launches the default shape instead, so the result equals the default
    shape's bit for bit."""
    torch = _torch()
    m, n0 = 32, 4
    prob = make_problem(0, prec, m, n0=n0, a=VELOCITY["mixed"][0], b=VELOCITY["mixed"][1])
    ctx = af.Context(prob)
    up_only = ctx.advance_shapes_upwind()
    assert up_only, "no upwind-only shape compiled for this case"
    assert set(up_only) <= set(ctx.advance_shapes())
    data = afsynth.fourier_modes(6)
    N = n0 * m
    d0 = afsynth.dofs_periodic(data, N, N, nq=4)
    blk = afsynth.periodic_to_blocks(d0, m)
    blocks = [{kk: blk[kk][p] for kk in KINDS} for p in range(n0 * n0)]
    dt = VELOCITY["mixed"][2] / (N * max(abs(prob.a), abs(prob.b)))
    out = []
    for shape in (up_only[-1], None):
        c = af.Context(prob)
        if shape is not None:
            c.set_advance_shape(*shape)
        h = af.Hierarchy(c, afsynth.uniform_leaves(n0, n0, 0))
        b0 = af.blocks_to_state(c, blocks)
        bufs = [b0, torch.zeros_like(b0)]
        mask = c.level_advance(h, bufs, 0, 0, dt, 7)
        torch.cuda.synchronize()
        out.append(bufs[mask & 1].cpu())
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("eq,prec,m,k,nt,vel", _shape_cases())
def test_level_advance_matches_oracle(eq, prec, m, k, nt, vel):
    """Temporally blocked level advance (K steps per launch, halo gathered
    from the neighbours' interiors) against the oracle's single periodic grid,
    with a step count that is not a multiple of K (tail launches)."""
    torch = _torch()
    print(f"[gpu-parity] level_advance eq={eq} prec={prec} m={m} K={k} NT={nt} velocity={vel}", flush=True)
    n0 = 4 if m <= 32 else 2
    phys = dict(a=VELOCITY[vel][0], b=VELOCITY[vel][1]) if eq == 0 else PHYS[eq]
    prob = make_problem(eq, prec, m, n0=n0, **phys)
    ctx = af.Context(prob)
    ctx.set_advance_shape(k, nt)
    data = afsynth.fourier_modes(6) if eq == 0 else afsynth.gaussian_pulse(6)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    N = n0 * m
    d0 = afsynth.dofs_periodic(data, N, N, nq=4)
    if prec == af.FP32:
        d0 = {kk: (v.astype(np.float32).astype(np.float64) if isinstance(v, np.ndarray) else v)
              for kk, v in d0.items()}
    blk = afsynth.periodic_to_blocks(d0, m)
    blocks = [{kk: blk[kk][p] for kk in KINDS} for p in range(n0 * n0)]
    h = af.Hierarchy(ctx, leaves)
    b0 = af.blocks_to_state(ctx, blocks)
    bufs = [b0, torch.zeros_like(b0)]
    nsteps = 2 * k + 1
    dt = VELOCITY[vel][2] / (N * max(abs(prob.a), abs(prob.b))) if eq == 0 else 0.4 / (N * prob.c)
    mask = ctx.level_advance(h, bufs, 0, 0, dt, nsteps)
    torch.cuda.synchronize()
    got = af.state_to_blocks(ctx, bufs[mask & 1])
    ref = oracle.run_periodic(eq, d0, dt, nsteps, a=prob.a, b=prob.b, c=prob.c)
    g = periodic_interior(got, leaves, m, n0)
    # FP64: per component, relative to the component's own maximum.  FP32:
    # relative to the maximum over all components, since every component
    # enters each acoustic node stencil and FP32 rounding scales with the
    # state, not with a component that starts at zero (the pulse's velocity);
    # a few units of FP32 rounding (6e-8) per step, at least 2e-6.
    scale = max(np.abs(ref[kk][q]).max() for kk in KINDS for q in range(prob.ncomp))
    for q in range(prob.ncomp):
        if prec == af.FP64:
            den, tol = max(np.abs(ref[kk][q]).max() for kk in KINDS), FP64_TOL
        else:
            den, tol = scale, max(2e-6, 3e-7 * nsteps)
        err = max(np.abs(g[kk][q] - ref[kk][q]).max() for kk in KINDS) / den
        assert err <= tol, (q, err)


def test_level_advance_rejects_mixed_levels():
    torch = _torch()
    n0, lmax, leaves = _amr_layouts()["diagonal"]
    ctx = af.Context(make_problem(0, af.FP64, 8, n0=n0, lmax=lmax))
    h = af.Hierarchy(ctx, leaves)
    b = ctx.new_state(len(leaves))
    with pytest.raises(af.AFError) as e:
        ctx.level_advance(h, [b, torch.zeros_like(b)], 0, 0, 0.001, 2)
    assert e.value.status == af._lib.AF_ERR_STATE


def test_single_patch_periodic_return_config1():
    """One 64x64 periodic patch, T = 2 (exact periodic return), FP64."""
    m, N = 64, 64
    prob = make_problem(0, af.FP64, m, n0=1, a=1.0, b=0.5)
    ctx = af.Context(prob)
    data = afsynth.sinsin_bump()
    leaves = [(0, 0, 0)]
    blocks = leaf_blocks(prob, leaves, data)
    nst = 5 * N
    got, _ = _uniform_run_gpu(ctx, prob, leaves, blocks, 0.4 / N, nst, "graph")
    d0 = afsynth.dofs_periodic(data, N, N, nq=6)
    ref = oracle.run_periodic(0, d0, 0.4 / N, nst, a=1.0, b=0.5)
    g = periodic_interior(got, leaves, m, 1)
    err = max(np.abs(g[k][0] - ref[k][0]).max() for k in KINDS) / np.abs(ref["avg"][0]).max()
    assert err <= FP64_TOL, err
    # exact return: the error against q0 is the method's, ~1e-2 at N=64
    e_exact = np.abs(g["avg"][0] - d0["avg"][0]).mean()
    assert 1e-4 < e_exact < 1e-3


def _amr_layouts():
    corner = [(0, ix, iy) for iy in range(4) for ix in range(4) if (ix, iy) != (1, 1)]
    corner += [(1, 2 + (q & 1), 2 + (q >> 1)) for q in range(4)]
    # three levels: the central 2x2 level-0 block refined once, and the
    # central 2x2 of that refined once more (2:1 balanced, also periodically)
    three = [(0, ix, iy) for iy in range(4) for ix in range(4) if not (1 <= ix <= 2 and 1 <= iy <= 2)]
    three += [(1, ix, iy) for iy in range(2, 6) for ix in range(2, 6) if not (3 <= ix <= 4 and 3 <= iy <= 4)]
    three += [(2, ix, iy) for iy in range(6, 10) for ix in range(6, 10)]
    return {"diagonal": (4, 1, afsynth.diagonal_leaves(4, 0)),
            "corner": (4, 1, afsynth.sort_leaves(corner)),
            "three": (4, 2, afsynth.sort_leaves(three))}


@pytest.mark.parametrize("layout", ["diagonal", "corner", "three"])
@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("tmin,smin", [(0, 0), (1, 1)])
def test_ghost_fill_parity(layout, eq, tmin, smin):
    """Random DOFs on an AMR hierarchy; the GPU fill must reproduce the
    oracle's fill of every ghost DOF (same-level, fine->coarse, coarse->fine,
    fine-wins nodes)."""
    torch = _torch()
    n0, lmax, leaves = _amr_layouts()[layout]
    print(f"[gpu-parity] fill {layout} eq={eq} tmin={tmin}", flush=True)
    m = 8
    rng = np.random.default_rng(5)
    prob = make_problem(eq, af.FP64, m, n0=n0, lmax=lmax, **PHYS[eq])
    ctx = af.Context(prob)
    blocks = _rand_blocks(rng, len(leaves), prob.ncomp, m)
    h = af.Hierarchy(ctx, leaves)
    # split the levels over the two buffers to exercise the level mask
    mask = 0b10
    b0 = af.blocks_to_state(ctx, blocks)
    b1 = b0.clone()
    ctx.ghost_fill(h, [b0, b1], mask, tmin, smin)
    torch.cuda.synchronize()
    g0, g1 = af.state_to_blocks(ctx, b0), af.state_to_blocks(ctx, b1)
    got = [g1[k] if (mask >> leaves[k][0]) & 1 else g0[k] for k in range(len(leaves))]
    o = oracle.Hier(eq, m, n0, n0, lmax, a=prob.a, b=prob.b, c=prob.c)
    o.set_leaves(leaves)
    for k, b in enumerate(blocks):
        o.set_block(k, b)
    o.fill(tmin, smin)
    ref = oracle_blocks(o)
    err = rel_linf(got, ref, valid_masks(m))
    assert err.max() <= FP64_TOL, err


def _amr_run(eq, prec, leaves, n0, lmax, m, nsteps, data, use_graph):
    torch = _torch()
    prob = make_problem(eq, prec, m, n0=n0, lmax=lmax, **PHYS[eq])
    ctx = af.Context(prob)
    h = af.Hierarchy(ctx, leaves)
    blocks = leaf_blocks(prob, leaves, data)
    b0 = af.blocks_to_state(ctx, blocks)
    bufs = [b0, torch.zeros_like(b0)]
    reg = torch.zeros((len(leaves), 4, m, prob.ncomp), dtype=torch.float64, device="cuda")
    s_in = torch.zeros(prob.ncomp, dtype=torch.float64, device="cuda")
    s_out = torch.zeros_like(s_in)
    mask = 0
    ctx.ghost_fill(h, bufs, mask, 0, 0)
    ctx.reduce_sum(h, bufs, mask, s_in)
    dt0 = 0.4 * prob.dx(0) / (1.0 if eq == 0 else prob.c)
    for _ in range(nsteps):
        mask = ctx.amr_coarse_step(h, bufs, mask, dt0, reg, use_graph=use_graph)
    ctx.reduce_sum(h, bufs, mask, s_out)
    torch.cuda.synchronize()
    # scale of the conserved sums: sum |Q| * cell area over the leaves
    scale = np.zeros(prob.ncomp)
    for (l, _, _), b in zip(leaves, blocks):
        scale += np.abs(b["avg"][:, 2:2 + m, 2:2 + m]).sum(axis=(1, 2)) * prob.dx(l) * prob.dy(l)
    scale = np.full(prob.ncomp, scale.max())  # components starting at zero share the overall scale
    g0, g1 = af.state_to_blocks(ctx, bufs[0]), af.state_to_blocks(ctx, bufs[1])
    got = [g1[k] if (mask >> leaves[k][0]) & 1 else g0[k] for k in range(len(leaves))]
    assert float(reg.abs().max()) == 0.0  # registers are consumed each coarse step
    return got, s_in.cpu().numpy(), s_out.cpu().numpy(), scale, prob, dt0


@pytest.mark.parametrize("layout", ["diagonal", "three"])
@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("use_graph", [False, True])
def test_amr_coarse_step_parity_fp64(layout, eq, use_graph):
    """Subcycled coarse steps with the conservative fix (Sec. 3.2) against the
    oracle's recursion; also global conservation on the GPU."""
    n0, lmax, leaves = _amr_layouts()[layout]
    print(f"[gpu-parity] amr {layout} eq={eq} graph={use_graph}", flush=True)
    m, nsteps = 8, 3
    data = afsynth.fourier_modes(1) if eq == 0 else afsynth.gaussian_pulse(1)
    got, s_in, s_out, scale, prob, dt0 = _amr_run(eq, af.FP64, leaves, n0, lmax, m, nsteps, data, use_graph)
    o = oracle.Hier(eq, m, n0, n0, lmax, a=prob.a, b=prob.b, c=prob.c)
    o.set_leaves(leaves)
    for k, b in enumerate(leaf_blocks(prob, leaves, data)):
        o.set_block(k, b)
    o.run(dt0, nsteps)
    err = rel_linf(got, oracle_blocks(o), closed_masks(m))
    assert err.max() <= FP64_TOL, err
    assert (np.abs(s_out - s_in) <= 1e-13 * scale).all(), (s_in, s_out, scale)


@pytest.mark.parametrize("eq", [0, 1])
def test_amr_fp32_error_and_conservation(eq):
    """FP32 bulk with FP64 registers and sums: error against the FP64 oracle
    and conservation drift at FP32 round-off (stated bounds 1e-5 and 1e-6
    relative after 4 coarse steps)."""
    n0, lmax, leaves = _amr_layouts()["diagonal"]
    m, nsteps = 8, 4
    data = afsynth.fourier_modes(2) if eq == 0 else afsynth.gaussian_pulse(2)
    got, s_in, s_out, scale, prob, dt0 = _amr_run(eq, af.FP32, leaves, n0, lmax, m, nsteps, data, True)
    o = oracle.Hier(eq, m, n0, n0, lmax, a=prob.a, b=prob.b, c=prob.c)
    o.set_leaves(leaves)
    for k, b in enumerate(leaf_blocks(prob, leaves, data)):
        o.set_block(k, {kk: v.astype(np.float32).astype(np.float64) for kk, v in b.items()})
    o.run(dt0, nsteps)
    err = rel_linf(got, oracle_blocks(o), closed_masks(m))
    drift = (np.abs(s_out - s_in) / scale).max()
    print(f"[gpu-parity] fp32 amr eq={eq}: rel Linf vs oracle {err}, conservation drift {drift}", flush=True)
    assert err.max() < 1e-5
    assert drift < 1e-6


@pytest.mark.parametrize("eq,mode", [(1, af.TAG_GRADIENT), (0, af.TAG_MAXMIN)])
def test_tag_and_regrid_parity(eq, mode):
    """Tags (Sec. 3 criteria) from the GPU match the oracle's; applying them
    (refine, balance, coarsen, transfers of Sec. 3.1, full fill) on the GPU
    gives the oracle's new hierarchy and DOFs."""
    torch = _torch()
    m, n0, lmax = 8, 2, 3
    prob = make_problem(eq, af.FP64, m, n0=n0, lmax=lmax, **PHYS[eq])
    ctx = af.Context(prob)
    leaves = afsynth.diagonal_leaves(n0, 1)
    data = afsynth.gaussian_pulse(4) if eq == 1 else afsynth.fourier_modes(4)
    blocks = leaf_blocks(prob, leaves, data)
    h = af.Hierarchy(ctx, leaves)
    b0 = af.blocks_to_state(ctx, blocks)
    bufs = [b0, b0]
    ctx.ghost_fill(h, bufs, 0, 0, 0)
    o = oracle.Hier(eq, m, n0, n0, lmax, a=prob.a, b=prob.b, c=prob.c)
    o.set_leaves(leaves)
    for k, b in enumerate(blocks):
        o.set_block(k, b)
    o.fill()
    # thresholds halfway between distinct criterion values (no ties), so that
    # some patches refine and some families may coarsen
    _, v0 = o.tag(mode, 0, 1e300, -1.0)
    sv = np.unique(v0)
    tr = 0.5 * (sv[int(0.7 * len(sv))] + sv[int(0.7 * len(sv)) - 1])
    tc = 0.5 * (sv[int(0.5 * len(sv))] + sv[int(0.5 * len(sv)) - 1])
    tags = torch.zeros(len(leaves), dtype=torch.int8, device="cuda")
    vals = torch.zeros(len(leaves), dtype=torch.float64, device="cuda")
    ctx.regrid_tag(h, bufs, 0, mode, 0, tr, tc, tags, vals)
    otags, ovals = o.tag(mode, 0, tr, tc)
    torch.cuda.synchronize()
    np.testing.assert_allclose(vals.cpu().numpy(), ovals, rtol=1e-12)
    t_host = tags.cpu().numpy()
    np.testing.assert_array_equal(t_host, otags)
    assert (t_host == 1).any() and (t_host == -1).any()
    nh = h.regrid(t_host)
    dst = ctx.new_state(len(nh))
    ctx.regrid_apply(h, bufs, 0, nh, dst)
    ctx.ghost_fill(nh, [dst, dst], 0, 0, 0)
    torch.cuda.synchronize()
    o.regrid(otags)
    assert nh.leaves() == o.leaves()
    err = rel_linf(af.state_to_blocks(ctx, dst), oracle_blocks(o), valid_masks(m))
    assert err.max() <= FP64_TOL, err


@pytest.mark.parametrize("prec", [af.FP64, af.FP32])
def test_full_size_config2_sampled(prec):
    """The benchmark workload at full size: 16x16 patches of 32x32 cells
    (512^2), seeded 8-mode Fourier data, in the launch configuration the
    benchmark times (hipGraph coarse steps), 4 steps against the oracle's
    single 512^2 periodic grid."""
    print(f"[gpu-parity] full size config 2 prec={prec}", flush=True)
    m, n0, nsteps = 32, 16, 4
    N = m * n0
    prob = make_problem(0, prec, m, n0=n0, a=1.0, b=0.5)
    ctx = af.Context(prob)
    data = afsynth.fourier_modes(0)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    d0 = afsynth.dofs_periodic(data, N, N, nq=4)
    if prec == af.FP32:
        d0 = {k: (v.astype(np.float32).astype(np.float64) if isinstance(v, np.ndarray) else v)
              for k, v in d0.items()}
    blocks = afsynth.periodic_to_blocks(d0, m)
    blocks = [{k: blocks[k][p] for k in KINDS} for p in range(n0 * n0)]
    dt = 1.0 / 1280
    got, _ = _uniform_run_gpu(ctx, prob, leaves, blocks, dt, nsteps, "graph")
    ref = oracle.run_periodic(0, d0, dt, nsteps, a=1.0, b=0.5)
    g = periodic_interior(got, leaves, m, n0)
    err = max(np.abs(g[k][0] - ref[k][0]).max() for k in KINDS) / np.abs(ref["avg"][0]).max()
    print(f"[gpu-parity] full size config 2 prec={prec}: rel Linf {err}", flush=True)
    assert err <= (FP64_TOL if prec == af.FP64 else 2e-6), err


@pytest.mark.parametrize("prec", [af.FP64, af.FP32])
def test_full_size_config2_level_advance(prec):
    """The benchmark's timed path at full size: 16x16 patches of 32x32 cells
    (512^2), seeded 8-mode Fourier data, the autotuner's level-advance shape
    (as bench.py picks it), 2K + 1 steps (full launches and a tail) against
    the oracle's single 512^2 periodic grid, every DOF compared."""
    torch = _torch()
    m, n0 = 32, 16
    N = m * n0
    prob = make_problem(0, prec, m, n0=n0, a=1.0, b=0.5)
    ctx = af.Context(prob)
    data = afsynth.fourier_modes(0)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    d0 = afsynth.dofs_periodic(data, N, N, nq=4)
    if prec == af.FP32:
        d0 = {k: (v.astype(np.float32).astype(np.float64) if isinstance(v, np.ndarray) else v)
              for k, v in d0.items()}
    blocks = afsynth.periodic_to_blocks(d0, m)
    blocks = [{k: blocks[k][p] for k in KINDS} for p in range(n0 * n0)]
    h = af.Hierarchy(ctx, leaves)
    b0 = af.blocks_to_state(ctx, blocks)
    dt = 1.0 / 1280
    ctx.autotune(h, [b0.clone(), torch.zeros_like(b0)], 0, dt, reps=3)
    K, NT = ctx.advance_shape
    assert K > 0
    nsteps = 2 * K + 1
    print(f"[gpu-parity] full size config 2 level advance prec={prec} K={K} NT={NT} steps={nsteps}", flush=True)
    bufs = [b0, torch.zeros_like(b0)]
    mask = ctx.level_advance(h, bufs, 0, 0, dt, nsteps)
    torch.cuda.synchronize()
    got = af.state_to_blocks(ctx, bufs[mask & 1])
    ref = oracle.run_periodic(0, d0, dt, nsteps, a=1.0, b=0.5)
    g = periodic_interior(got, leaves, m, n0)
    err = max(np.abs(g[k][0] - ref[k][0]).max() for k in KINDS) / np.abs(ref["avg"][0]).max()
    print(f"[gpu-parity] full size config 2 level advance prec={prec}: rel Linf {err}", flush=True)
    # FP32: rounding accumulates step by step; about 5 units of FP32 rounding
    # (6e-8) per step (the 4-step general-path run measures 1.5e-7 per step)
    assert err <= (FP64_TOL if prec == af.FP64 else 3e-7 * nsteps), err


@pytest.mark.parametrize("prec", [af.FP32, af.FP64])
def test_level_advance_graph_replays_match_eager(prec):
    """The benchmark times the level advance as a captured HIP graph.  Three
    replays, each after eager work (a state reset and an eager run on the
    same buffers) and a synchronisation, must each equal the eager run bit
    for bit; the step count is not a multiple of K, so the graph also holds
    the tail launch."""
    torch = _torch()
    m, n0 = 32, 4
    prob = make_problem(0, prec, m, n0=n0, a=1.0, b=0.5)
    ctx = af.Context(prob)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    h = af.Hierarchy(ctx, leaves)
    init = af.blocks_to_state(ctx, leaf_blocks(prob, leaves, afsynth.fourier_modes(2), nq=4))
    K, NT = ctx.advance_shape
    nsteps = 3 * K + 1
    dt = 0.4 * prob.dx(0)
    bufs = [init.clone(), torch.zeros_like(init)]

    def reset():
        bufs[0].copy_(init)
        bufs[1].zero_()

    reset()
    mask_e = ctx.level_advance(h, bufs, 0, 0, dt, nsteps)
    torch.cuda.synchronize()
    eager = [b.clone() for b in bufs]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        mask_g = ctx.level_advance(h, bufs, 0, 0, dt, nsteps)
    assert mask_g == mask_e
    for rep in range(3):
        reset()
        ctx.level_advance(h, bufs, 0, 0, dt, K)  # eager work between replays
        torch.cuda.synchronize()
        reset()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(bufs, eager):
            assert torch.equal(a, b), rep


def test_fp32_benchmark_run_stays_near_fp64():
    """The whole benchmark run (512^2, 1280 steps to T = 1) in FP32 against
    the same run in FP64 (whose level advance is pinned to the oracle above).
    FP32 weights differ from the FP64 ones by rounding (6e-8 relative each).
    That perturbs the discrete operator, so the two runs separate linearly
    in time; the worst case is 1280 steps x sum|w| (1.76 for the composed
    average) x 6e-8 = 1.4e-4.  Rounding each stencil so that it still sums
    to exactly 1 removes the constant mode's share of it, which dominated:
    with plainly rounded weights the run ended 5.9e-5 away from FP64, and
    with unit-sum rounding it ends at 1.8e-5.  The bound, 5e-5, separates
    the two."""
    torch = _torch()
    m, n0 = 32, 16
    data = afsynth.fourier_modes(0)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    out = {}
    for prec in (af.FP64, af.FP32):
        prob = make_problem(0, prec, m, n0=n0, a=1.0, b=0.5)
        ctx = af.Context(prob)
        blocks = leaf_blocks(prob, leaves, data, nq=4)
        h = af.Hierarchy(ctx, leaves)
        b0 = af.blocks_to_state(ctx, blocks)
        bufs = [b0, torch.zeros_like(b0)]
        mask = ctx.level_advance(h, bufs, 0, 0, 1.0 / 1280, 1280)
        torch.cuda.synchronize()
        out[prec] = af.state_to_blocks(ctx, bufs[mask & 1])
    g64 = periodic_interior(out[af.FP64], leaves, m, n0)
    g32 = periodic_interior(out[af.FP32], leaves, m, n0)
    den = max(np.abs(g64[k][0]).max() for k in KINDS)
    err = max(np.abs(g32[k][0] - g64[k][0]).max() for k in KINDS) / den
    print(f"[gpu-parity] FP32 vs FP64 after 1280 steps: rel Linf {err:.3e}", flush=True)
    assert err <= 5e-5, err


@pytest.mark.parametrize("eq", [0, 1])
def test_fp32_constant_state_does_not_drift(eq):
    """A constant state under the FP32 level advance, 640 steps: with stencils
    that sum to exactly 1 (values) and 0 (gradients) the state may only
    wander by unbiased rounding, far below the 640 x 3e-8 = 2e-5 a biased
    weight sum gives."""
    torch = _torch()
    m, n0 = 16, 4
    prob = make_problem(eq, af.FP32, m, n0=n0, a=1.0, b=0.5, c=1.0)
    ctx = af.Context(prob)
    leaves = afsynth.uniform_leaves(n0, n0, 0)
    h = af.Hierarchy(ctx, leaves)
    t = ctx.new_state(len(leaves))
    t.fill_(0.7)
    bufs = [t, torch.zeros_like(t)]
    dt = 0.4 * prob.dx(0) / (1.0 if eq == 0 else prob.c) * (1.0 if eq == 0 else 0.5)
    mask = ctx.level_advance(h, bufs, 0, 0, dt, 640)
    torch.cuda.synchronize()
    got = af.state_to_blocks(ctx, bufs[mask & 1])
    g = periodic_interior(got, leaves, m, n0)
    comps = [0] if eq == 0 else [0, 1, 2]
    for q in comps:
        ref = 0.7
        err = max(np.abs(g[k][q] - ref).max() for k in KINDS) / ref
        print(f"[gpu-parity] FP32 constant state eq={eq} comp={q}: rel drift {err:.3e}", flush=True)
        assert err <= 2e-6, (q, err)


@pytest.mark.parametrize("prec", [af.FP32, af.FP64])
def test_fma_probe_computes_its_chains(prec):
    """The FMA rate probe runs real arithmetic: thread t's output is the sum
    over k < 8 of the recurrence x <- x a + b from x = t + k, 16 x iters
    times, recomputed here in FP64 (FP32 within its rounding)."""
    torch = _torch()
    iters, nblocks = 3, 2
    dt = torch.float32 if prec == af.FP32 else torch.float64
    out = torch.zeros(nblocks * 256, dtype=dt, device="cuda")
    af._lib.check(af._lib.load().af_fma_probe(int(prec), af._ptr(out), nblocks, iters, af._stream()))
    torch.cuda.synchronize()
    got = out.cpu().double().numpy()
    a, b = (0.999999, 1e-7)
    if prec == af.FP32:
        a, b = float(np.float32(a)), float(np.float32(b))
    t = np.arange(nblocks * 256) % 256
    ref = np.zeros_like(got)
    for k in range(8):
        x = (t + k).astype(np.float64)
        for _ in range(16 * iters):
            x = x * a + b
        ref += x
    # FP32: at most one rounding (2^-24 relative) per step of the 48-step chains
    tol = 1e-12 if prec == af.FP64 else 48 * 2.0 ** -24
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)) <= tol
    rate = af.fma_probe(prec, nblocks=512, iters=16)
    print(f"[gpu-parity] FMA probe prec={prec}: {rate:.1f} TFLOP/s", flush=True)
    assert rate > 1.0


def test_edge_cases_and_errors():
    torch = _torch()
    prob = make_problem(0, af.FP64, 16, n0=2, a=1.0, b=0.5)
    ctx = af.Context(prob)
    t = ctx.new_state(4)
    u = torch.zeros_like(t)
    ctx.patch_step(t, u, 0, 0, 0, 0.01, 0)  # empty range: nothing launched
    with pytest.raises(af.AFError) as e:
        ctx.patch_step(t, u, 0, 4, 0, 2.0 * prob.dx(0), 0)
    assert e.value.status == af._lib.AF_ERR_CFL
    with pytest.raises(af.AFError) as e:
        ctx.patch_step(t, t, 0, 4, 0, 0.01, 0)
    assert e.value.status == af._lib.AF_ERR_ARG
    with pytest.raises(af.AFError) as e:
        ctx.patch_step(t, u, 2, 4, 0, 0.01, 0)
    assert e.value.status == af._lib.AF_ERR_LAYOUT
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0.0


def test_autotune_without_level_advance_shape():
    """A level whose leaves all have same-level neighbours but no compiled
    level-advance shape (acoustics, FP64, m = 32): the autotuner still tunes
    the patch step and reports -1 for the level advance."""
    torch = _torch()
    n0, m = 2, 32
    prob = make_problem(1, af.FP64, m, n0=n0)
    ctx = af.Context(prob)
    assert ctx.advance_shapes() == []
    h = af.Hierarchy(ctx, afsynth.uniform_leaves(n0, n0, 0))
    b = ctx.new_state(n0 * n0)
    step_us, adv_us = ctx.autotune(h, [b, torch.zeros_like(b)], 0, 0.4 / (n0 * m), reps=1)
    assert step_us > 0 and adv_us == -1
