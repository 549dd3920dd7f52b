"""Benchmark: batched Active Flux patch step on one MI355X.

Workload (the metric's configuration): 2D linear advection, a=1, b=0.5, on
the periodic unit square as one level of 16x16 patches of 32x32 cells
(512^2 cells, two ghost layers), seeded 8-mode Fourier initial data, T=1
(1280 steps at CFL 0.4).  One "step" is one pass of the whole path: ghost
fill between patches plus the patch step of every patch, replayed as a
hipGraph.  FP32 is the headline (FP32 state and arithmetic, FP64 sums); the
FP64 path is timed beside it.

Prints one JSON line.  --gpus N with N > 1 is not supported (single GPU).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M, N0 = 32, 16
NCELL = (M * N0) ** 2
T_FINAL = 1.0
NSTEPS_T = 1280
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the level-advance kernel (k_level_advance_up) on
# this workload, from rocprofv3 FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00 (scales
# from a plain 64 MiB copy), keyed by (precision, K, threads); valid only for
# the kernel source the counters were taken on
# (profiles/k_level_advance_up_512sq.md holds the commands).
PROFILED_TRAFFIC = {
    ("fp32", 1, 256): 10.26e6, ("fp32", 2, 256): 10.37e6, ("fp32", 2, 512): 10.33e6, ("fp32", 4, 512): 10.52e6,
    ("fp32", 4, 1024): 10.49e6, ("fp32", 5, 512): 10.61e6, ("fp32", 5, 1024): 10.58e6,
    ("fp32", 6, 512): 10.70e6, ("fp32", 6, 768): 10.68e6, ("fp32", 6, 1024): 10.68e6,
    ("fp32", 7, 1024): 10.76e6, ("fp32", 8, 512): 10.94e6, ("fp32", 8, 1024): 10.85e6,
    ("fp32", 10, 512): 11.13e6, ("fp32", 10, 1024): 11.03e6, ("fp32", 12, 512): 11.33e6,
    ("fp32", 12, 1024): 11.21e6, ("fp32", 14, 1024): 11.39e6, ("fp32", 16, 1024): 11.57e6,
    ("fp32", 18, 1024): 11.75e6, ("fp32", 20, 1024): 11.93e6,
    ("fp64", 1, 256): 19.77e6, ("fp64", 2, 512): 19.87e6, ("fp64", 3, 1024): 20.02e6, ("fp64", 4, 512): 20.21e6,
    ("fp64", 4, 1024): 20.19e6, ("fp64", 5, 1024): 20.35e6, ("fp64", 6, 1024): 20.52e6,
    ("fp64", 8, 1024): 20.85e6, ("fp64", 10, 1024): 21.18e6, ("fp64", 12, 1024): 21.51e6,
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=NSTEPS_T)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-steps", type=int, default=144)
    p.add_argument("--general-steps", type=int, default=128)
    p.add_argument("--no-amr", action="store_true", help="skip the adaptive acoustics runs")
    p.add_argument("--sweep", action="store_true",
                   help="roofline sweep: uniform grids up to 4096^2 (HBM resident); one JSON line per case")
    p.add_argument("--copy-probe", action="store_true",
                   help="only run a plain 64 MiB device copy 20 times (HBM counter calibration)")
    p.add_argument("--peak-probe", action="store_true",
                   help="only measure the device's copy bandwidth and vector FMA rate (one JSON line)")
    p.add_argument("--only", choices=["amr", "rotation", "swirl", "burgers"],
                   help="only run one workload block (one JSON line with that block), e.g. for a profiler")
    return p.parse_args()


def peak_probe():
    """Copy bandwidth (device-to-device copy of 1 GiB, read + write bytes)
    and the vector FMA rate in FP32 and FP64 (af_fma_probe), to set beside
    the published peaks the roofline fractions use."""
    import torch
    import paper_2205_07572_amd as af
    n = 1 << 28  # 1 GiB of float32
    a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(10):
        ms, _ = _event_ms(lambda: b.copy_(a))
        best = min(best, ms)
    copy_gbs = 2 * 4 * n / (best * 1e-3) / 1e9
    fma = {name: max(af.fma_probe(prec) for _ in range(5)) for name, prec in (("fp32", af.FP32), ("fp64", af.FP64))}
    print(json.dumps({"peak_probe": True, "copy_gbs": copy_gbs, "copy_frac_of_8000": copy_gbs / HBM_PEAK_GBS,
                      "fma_tflops": fma, "published_tflops": PEAK_TFLOPS,
                      "note": "FP32 kernels are compiled without packed FP32 instructions"}), flush=True)


def copy_probe():
    """A plain device-to-device copy of known size: FETCH_SIZE / WRITE_SIZE
    of this kernel calibrate the counters against bytes actually moved."""
    import torch
    n = 64 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 20}), flush=True)


def setup(prec, data):
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    prob = af.Problem(eq=af.ADVECTION, prec=prec, m=M, n0x=N0, n0y=N0, lmax=0, a=1.0, b=0.5)
    ctx = af.Context(prob)
    leaves = afsynth.uniform_leaves(N0, N0, 0)
    blocks = []
    for (l, ix, iy) in leaves:
        dx = prob.dx(0)
        blocks.append(afsynth.dofs_block(data, M, 2, ix * M * dx, iy * M * dx, dx, dx, 4))
    h = af.Hierarchy(ctx, leaves)
    b0 = af.blocks_to_state(ctx, blocks)
    bufs = [b0, torch.zeros_like(b0)]
    reg = torch.zeros((len(leaves), 4, M, 1), dtype=torch.float64, device="cuda")
    return ctx, h, bufs, reg, blocks


def run_steps(ctx, h, bufs, reg, mask, nsteps, dt):
    for _ in range(nsteps):
        mask = ctx.amr_coarse_step(h, bufs, mask, dt, reg, use_graph=True)
    return mask


def _event_ms(fn):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


def time_path(prec, data, steps, warmup, dt, general_steps):
    """Autotune, then time `steps` steps of the level advance (the path this
    workload takes: ghost exchange by gathering from same-level neighbours,
    K steps per launch) and, for reference, `general_steps` coarse steps of
    the general path (af_ghost_fill + af_patch_step replayed as a hipGraph)."""
    import torch
    import paper_2205_07572_amd as af
    ctx, h, bufs, reg, blocks = setup(prec, data)
    init = af.blocks_to_state(ctx, blocks)

    def reset():
        bufs[0].copy_(init)
        bufs[1].zero_()
        torch.cuda.synchronize()

    step_us, adv_us = ctx.autotune(h, bufs, 0, dt, reps=10)
    K, NT = ctx.advance_shape
    reset()
    ctx.level_advance(h, bufs, 0, 0, dt, warmup)
    torch.cuda.synchronize()
    reset()
    eager_ms, _ = _event_ms(lambda: ctx.level_advance(h, bufs, 0, 0, dt, steps))
    # The timed run replays the same launches captured once as a HIP graph
    # (torch's capture of the library's launches on its stream; nothing runs
    # during capture).  A replay issues the whole sequence without the host
    # in between launches.
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        mask = ctx.level_advance(h, bufs, 0, 0, dt, steps)
    reset()
    graph.replay()  # untimed warm replay
    torch.cuda.synchronize()
    reset()
    ms, _ = _event_ms(lambda: graph.replay())
    out = af.state_to_blocks(ctx, bufs[mask & 1])
    # dominant kernel: one level-advance launch of K steps, in the
    # benchmark's launch configuration, timed with HIP events on the stream
    # it runs on: nl launches of K steps, captured and replayed like the
    # timed run.
    nl = 200
    g_nl = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_nl):
        ctx.level_advance(h, bufs, 0, 0, dt, K * nl)
    g_nl.replay()
    torch.cuda.synchronize()
    k_sep, _ = _event_ms(lambda: g_nl.replay())
    k_sep /= nl
    # the roofline uses the average launch of the timed region itself when
    # it consists of whole K-step launches (steps a multiple of K)
    k_ms = ms / (steps // K) if steps % K == 0 else k_sep
    # general path for reference
    reset()
    run_steps(ctx, h, bufs, reg, 0, 4, dt)
    torch.cuda.synchronize()
    reset()
    g_ms, _ = _event_ms(lambda: run_steps(ctx, h, bufs, reg, 0, general_steps, dt))
    return dict(ms=ms, eager_ms=eager_ms, k_ms=k_ms, k_sep=k_sep, K=K, NT=NT, out=out, tile=ctx.tile, step_us=step_us, adv_us=adv_us,
                general_ms_per_step=g_ms / general_steps)


# FP32 / FP64 vector peaks (MI355X published figures, TFLOP/s); packed FP32
# instructions are disabled in this build, so FP32 kernels can reach at most
# half of the FP32 figure.
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
# algorithmic flops per cell-update of the collapsed stencils: advection 6
# node values x 9 FMA + 3 time sums (2 ops) + 4 face sums (2 ops) + update
# (6 ops); acoustics: corner 25-entry, x- and y-edge 15-entry stencils, each
# with 7 dot products at 2 time levels (770 FMA), + 9 time sums + 12 face
# sums x 2 + 3-component update (about 24 ops)
FLOPS_PER_UPDATE = {0: 2 * 54 + 6 + 8 + 6, 1: 2 * 770 + 18 + 24 + 24}


def sweep():
    """Roofline sweep on uniform periodic grids from 1024^2 to 4096^2 cells
    (state up to 6.3 GB per buffer, far beyond the 256 MB Infinity Cache):
    advection and acoustics, 32^2 and 16^2 patches, FP32 and FP64.  Launch
    times come from the autotuner, which times back-to-back launches of
    every kernel shape with HIP events on the stream they run on.  State
    values are random (timing does not depend on them).  One JSON line per
    case."""
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    cases = [(0, 32, 1024), (0, 32, 2048), (0, 32, 4096), (0, 16, 4096),
             (1, 16, 1024), (1, 16, 2048), (1, 16, 4096), (1, 32, 4096)]
    for eq, m, N in cases:
        n0 = N // m
        for name, prec, wb in (("fp32", af.FP32, 4), ("fp64", af.FP64, 8)):
            phys = dict(a=1.0, b=0.5) if eq == 0 else dict(c=1.0)
            prob = af.Problem(eq=eq, prec=prec, m=m, n0x=n0, n0y=n0, lmax=0, **phys)
            ctx = af.Context(prob)
            h = af.Hierarchy(ctx, afsynth.uniform_leaves(n0, n0, 0))
            t = ctx.new_state(n0 * n0)
            g = torch.Generator(device="cuda").manual_seed(N + m + eq)
            t.copy_(torch.randn(t.shape, generator=g, device="cuda", dtype=t.dtype))
            bufs = [t, torch.zeros_like(t)]
            dt = (0.4 if eq == 0 else 0.4) / N
            step_us, adv_us = ctx.autotune(h, bufs, 0, dt, reps=10)
            ncomp = 1 if eq == 0 else 3
            alg = 8 * ncomp * wb * N * N  # algorithmic bytes per step
            flops = FLOPS_PER_UPDATE[eq] * N * N
            line = {"sweep": True, "equation": ["advection", "acoustics"][eq], "patch": m, "cells": N * N,
                    "prec": name, "state_bytes_per_buffer": t.numel() * wb,
                    "patch_step": {"tile_rows": ctx.tile, "launch_us": step_us,
                                   "gbs": alg / (step_us * 1e-6) / 1e9,
                                   "hbm_frac": alg / (step_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                   "alu_frac": flops / (step_us * 1e-6) / 1e12 / PEAK_TFLOPS[name],
                                   "cell_updates_per_s": N * N / (step_us * 1e-6)}}
            if adv_us > 0:
                K, NT = ctx.advance_shape
                line["level_advance"] = {"K": K, "threads": NT, "launch_us": adv_us * K,
                                         "gbs": alg / (adv_us * 1e-6) / 1e9,
                                         "hbm_frac": alg / (adv_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                         "alu_frac": flops / (adv_us * 1e-6) / 1e12 / PEAK_TFLOPS[name],
                                         "cell_updates_per_s": N * N / (adv_us * 1e-6)}
            print(json.dumps(line), flush=True)
            del bufs, t
            torch.cuda.empty_cache()


def amr_runs():
    """Adaptive acoustics, the two AMR workloads, FP32 bulk and FP64, to
    T = 0.5 with plain gradient tagging every 4 coarse steps:
      config3: Gaussian pulse exp(-200 |x - x0|^2), 3 levels, refine at
               |grad p| >= 1, coarsen below 0.25;
      config4: wave packet exp(-50 |x - x0|^2) cos(k.x), |k| = 80 pi, 4
               levels, refine at 8, coarsen below 2.
    Base 8x8 patches of 16^2, CFL 0.4 on every level (subcycling), seed 0.
    Cell-updates/s counts step time only (device events around the coarse
    steps); time to solution includes the regrids.  The error is the
    L-infinity error of the pressure averages over all leaves against the
    exact Fourier solution."""
    import math
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    specs = {"config3": (2, afsynth.gaussian_pulse(0), lambda d: afsynth.gaussian_pulse_exact(d, 200.0),
                         TagRule(af.TAG_GRADIENT, 0, 1.0, 0.25)),
             "config4": (3, afsynth.wave_packet(0), afsynth.wave_packet_exact, TagRule(af.TAG_GRADIENT, 0, 8.0, 2.0))}
    T, every, m = 0.5, 4, 16
    out = {}
    for name, (lmax, data, exact_of, rule) in specs.items():
        exact = exact_of(data)
        res = {}
        for pname, prec in (("fp32", af.FP32), ("fp64", af.FP64)):
            prob = af.Problem(eq=af.ACOUSTICS, prec=prec, m=m, n0x=8, n0y=8, lmax=lmax, c=1.0)

            def block_fn(l, ix, iy, prob=prob):
                dx = prob.dx(l)
                return afsynth.dofs_block(data, m, 2, ix * m * dx, iy * m * dx, dx, dx, 4)

            run = initial_hierarchy(prob, block_fn, rule)
            n = math.ceil(T / (0.4 * prob.dx(0)))
            dt0 = T / n
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step = 0
            while step < n:
                k = min(every, n - step)
                run.coarse_steps(dt0, k)
                step += k
                if step < n:
                    run.regrid(rule)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            leaves = run.hier.leaves()
            blocks = run.blocks()
            err = 0.0
            for l in sorted({lv for lv, _, _ in leaves}):
                dx = prob.dx(l)
                nl = 8 * m << l
                xs = (np.arange(nl) + 0.5) * dx
                E = exact.grid_values(xs, xs, T, dx, dx)[0]  # [y][x] pressure averages
                for b, (lv, ix, iy) in zip(blocks, leaves):
                    if lv == l:
                        d = b["avg"][0, 2:2 + m, 2:2 + m] - E[iy * m:(iy + 1) * m, ix * m:(ix + 1) * m]
                        err = max(err, float(np.abs(d).max()))
            st = run.stats
            hist = st.leaves_history
            res[pname] = {"coarse_steps": st.coarse_steps, "regrids": st.regrids,
                          "cell_updates": st.cell_updates, "step_s": st.step_seconds,
                          "cell_updates_per_s": st.cell_updates / st.step_seconds,
                          "us_per_coarse_step": 1e6 * st.step_seconds / st.coarse_steps,
                          "regrid_s": st.regrid_seconds, "time_to_solution_s": wall,
                          "leaves_mean": float(np.mean(hist)) if hist else len(leaves), "leaves_max": max(hist or [0]),
                          "leaves_per_level_final": np.bincount([lv for lv, _, _ in leaves]).tolist(),
                          "linf_p_vs_exact": err}
            print(f"[bench] {name} {pname}: {st.coarse_steps} coarse steps, {res[pname]['cell_updates_per_s']:.3e} "
                  f"cell-updates/s, {res[pname]['us_per_coarse_step']:.0f} us/coarse step, leaves "
                  f"{res[pname]['leaves_mean']:.0f} (max {res[pname]['leaves_max']}), time to solution {wall:.3f} s, "
                  f"L-inf p {err:.3e}", file=sys.stderr, flush=True)
            del run
            torch.cuda.empty_cache()
        out[name] = res
    return out


def rotation_runs():
    """Solid-body rotation (a = -pi y, b = pi x on [-1, 1]^2, the smoothed
    disc of the advection test centred at (0.5, 0.5)), uniform levels 6 and 7
    (1024^2 and 2048^2 as 32^2 patches) to a half rotation at Courant number
    0.6 of the largest axis speed: cell-updates/s of the general path
    (ghost fill + patch step per step) in FP64 and FP32, and the L1 error of
    the averages (area-weighted, divided by the domain area) next to the
    paper's Table 2 values."""
    import math
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    m, T, omega = 32, 1.0, math.pi
    paper = {6: 4.599185e-06, 7: 5.826258e-07}
    data = afsynth.solid_body(afsynth.disc_q0(0.15, 0.02, 0.5, 0.5), omega)
    out = {}
    for level in (6, 7):
        N = 16 << level
        n0 = N // m
        d0 = afsynth.dofs_periodic(data, N, N, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, nq=4)
        blk = afsynth.periodic_to_blocks(d0, m)
        ex = afsynth.dofs_periodic(afsynth.InitialData(1, lambda x, y: data.exact(x, y, T)), N, N, x0=-1.0,
                                   y0=-1.0, lx=2.0, ly=2.0, nq=4)["avg"][0]
        dx = 2.0 / N
        n = math.ceil(T / (0.6 * dx / omega))
        res = {}
        for pname, prec in (("fp64", af.FP64), ("fp32", af.FP32)):
            prob = af.Problem(eq=af.ROTATION, prec=prec, m=m, n0x=n0, n0y=n0, lmax=0, x0=-1.0, y0=-1.0, lx=2.0,
                              ly=2.0, omega=omega)
            ctx = af.Context(prob)
            leaves = afsynth.uniform_leaves(n0, n0, 0)
            h = af.Hierarchy(ctx, leaves)
            b0 = af.blocks_to_state(ctx, [{k: blk[k][p] for k in af.KINDS} for p in range(n0 * n0)])
            bufs = [b0, torch.zeros_like(b0)]
            reg = torch.zeros((len(leaves), 4, m, 1), dtype=torch.float64, device="cuda")
            ctx.autotune(h, [b0.clone(), torch.zeros_like(b0)], 0, T / n, reps=3)
            mask = 0
            ms, mask = _event_ms(lambda: _rot_steps(ctx, h, bufs, reg, n, T / n))
            got = af.state_to_blocks(ctx, bufs[mask & 1])
            avg = np.zeros((N, N))
            for p, (_, ix, iy) in enumerate(leaves):
                avg[iy * m:(iy + 1) * m, ix * m:(ix + 1) * m] = got[p]["avg"][0, 2:2 + m, 2:2 + m]
            l1 = float(np.abs(avg - ex).sum() * dx * dx / 4.0)
            res[pname] = {"steps": n, "ms": ms, "cell_updates_per_s": N * N * n / (ms * 1e-3), "l1": l1,
                          "l1_over_paper": l1 / paper[level]}
            print(f"[bench] rotation level {level} ({N}^2) {pname}: {n} steps in {ms:.1f} ms, "
                  f"{res[pname]['cell_updates_per_s']:.3e} cell-updates/s, L1 {l1:.4e} "
                  f"({res[pname]['l1_over_paper']:.3f} x Table 2)", file=sys.stderr, flush=True)
            del bufs, b0
            torch.cuda.empty_cache()
        out[f"level{level}"] = res
    out["eoc_fp64"] = math.log2(out["level6"]["fp64"]["l1"] / out["level7"]["fp64"]["l1"])
    out["paper_eoc"] = 2.9807
    return out


def swirl_runs():
    """Swirl flow of Sec. 4.3 (Psi = sin^2(pi x) sin^2(pi y) cos(pi t) / pi on
    the periodic unit square, the two Gaussians of eq. id_swirl) to t = 1 at
    Courant number 0.6 of the largest speed (1): uniform levels 4, 5 and 6
    (256^2 to 1024^2 cells as 32^2 patches) in FP64 and FP32, and the
    diagonal refinement 3-4 (128^2 with the diagonal patches at 256^2, 16^2
    patches) with subcycling and with global time stepping.  Reports
    cell-updates/s of the general path (ghost fill + patch step per step) and
    the L1 error of the averages against the initial data (the exact solution
    at t = 1), next to the paper's Table 3."""
    import math
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    paper = {4: 5.722927e-06, 5: 7.268088e-07}
    data = afsynth.swirl_gaussians()
    out = {}

    def run(prec, m, n0, lmax, leaves, n, dt, global_step):
        prob = af.Problem(eq=af.SWIRL, prec=prec, m=m, n0x=n0, n0y=n0, lmax=lmax)
        ctx = af.Context(prob)
        h = af.Hierarchy(ctx, leaves)
        blocks = []
        for (l, ix, iy) in leaves:
            dx = prob.dx(l)
            blocks.append(afsynth.dofs_block(data, m, 2, ix * m * dx, iy * m * dx, dx, dx, 4))
        b0 = af.blocks_to_state(ctx, blocks)
        bufs = [b0, torch.zeros_like(b0)]
        reg = torch.zeros((len(leaves), 4, m, 1), dtype=torch.float64, device="cuda")
        ctx.ghost_fill(h, bufs, 0, 0, 0)
        warm, wm = [b0.clone(), torch.zeros_like(b0)], 0
        for k in range(2):  # untimed warm-up on a copy
            wm = ctx.amr_coarse_step(h, warm, wm, dt, reg, t0=k * dt, global_step=global_step)
        del warm

        def steps():
            mask = 0
            for k in range(n):
                mask = ctx.amr_coarse_step(h, bufs, mask, dt, reg, t0=k * dt, global_step=global_step)
            return mask

        ms, mask = _event_ms(steps)
        got = af.state_to_blocks(ctx, bufs[0]), af.state_to_blocks(ctx, bufs[1])
        l1, updates = 0.0, 0
        for k, (l, ix, iy) in enumerate(leaves):
            b = got[(mask >> l) & 1][k]["avg"][0, 2:2 + m, 2:2 + m]
            l1 += float(np.abs(b - blocks[k]["avg"][0, 2:2 + m, 2:2 + m]).sum()) * prob.dx(l) ** 2
            updates += m * m * n * (1 if global_step else 1 << l)
        del bufs, b0
        torch.cuda.empty_cache()
        return ms, l1, updates

    for level in (4, 5, 6):
        N, m = 16 << level, 32
        n0 = N // m
        n = math.ceil(1.0 / (0.6 / N))
        res = {}
        for pname, prec in (("fp64", af.FP64), ("fp32", af.FP32)):
            ms, l1, upd = run(prec, m, n0, 0, afsynth.uniform_leaves(n0, n0, 0), n, 1.0 / n, False)
            res[pname] = {"steps": n, "ms": ms, "cell_updates_per_s": upd / (ms * 1e-3), "l1": l1}
            if level in paper:
                res[pname]["l1_over_paper"] = l1 / paper[level]
            print(f"[bench] swirl level {level} ({N}^2) {pname}: {n} steps in {ms:.1f} ms, "
                  f"{res[pname]['cell_updates_per_s']:.3e} cell-updates/s, L1 {l1:.4e}", file=sys.stderr,
                  flush=True)
        out[f"level{level}"] = res
    out["eoc_4_5_fp64"] = math.log2(out["level4"]["fp64"]["l1"] / out["level5"]["fp64"]["l1"])
    out["paper_eoc_4_5"] = 2.9771
    m, n0 = 16, 8  # level 3 = 128^2 cells
    leaves = afsynth.diagonal_leaves(n0, 0)
    for mode, glob in (("subcycled", False), ("global", True)):
        n = math.ceil(1.0 / (0.6 / (n0 * m * (2 if glob else 1))))
        ms, l1, upd = run(af.FP64, m, n0, 1, leaves, n, 1.0 / n, glob)
        out[f"diag3_4_{mode}_fp64"] = {"steps": n, "ms": ms, "cell_updates_per_s": upd / (ms * 1e-3), "l1": l1}
        print(f"[bench] swirl diagonal 3-4 {mode}: {n} coarse steps in {ms:.1f} ms, L1 {l1:.4e}", file=sys.stderr,
              flush=True)
    out["paper_amr_3_4"] = {"subcycled": 5.758274e-06, "global": 5.724930e-06}
    out["adaptive"] = swirl_adaptive_runs(data)
    return out


def swirl_adaptive_runs(data):
    """Adaptive swirl runs (Table 3, rows 3-4 and 3-5): base level 3
    (8x8 patches of 16^2 = 128^2 cells), a patch refined where max - min of
    its averages exceeds 0.001 (the criterion of Sec. 4.1) and coarsened below
    it, regridded every coarse step (every 2^lmax global steps), FP64, to
    t = 1 with CFL 0.6 on every level.  L1 error of the leaf averages against
    the initial data (the exact solution at t = 1)."""
    import math
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    paper = {"subcycled": {1: 5.758274e-06, 2: 7.346642e-07}, "global": {1: 5.724930e-06, 2: 7.305236e-07}}
    rule = TagRule(af.TAG_MAXMIN, 0, 1e-3, 1e-3)
    m, n0 = 16, 8
    out = {}
    for lmax in (1, 2):
        for mode in ("subcycled", "global"):
            glob = mode == "global"
            prob = af.Problem(eq=af.SWIRL, prec=af.FP64, m=m, n0x=n0, n0y=n0, lmax=lmax)

            def block_fn(l, ix, iy, prob=prob):
                dx = prob.dx(l)
                return afsynth.dofs_block(data, m, 2, ix * m * dx, iy * m * dx, dx, dx, 4)

            run = initial_hierarchy(prob, block_fn, rule)
            n = math.ceil(1.0 / (0.6 * prob.dx(lmax if glob else 0)))
            dt, every = 1.0 / n, (1 << lmax) if glob else 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step = 0
            while step < n:
                k = min(every, n - step)
                run.coarse_steps(dt, k, global_step=glob)
                step += k
                if step < n:
                    run.regrid(rule)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            l1 = 0.0
            for b, (l, ix, iy) in zip(run.blocks(), run.hier.leaves()):
                ex = block_fn(l, ix, iy)["avg"][0, 2:2 + m, 2:2 + m]
                l1 += float(np.abs(b["avg"][0, 2:2 + m, 2:2 + m] - ex).sum()) * prob.dx(l) ** 2
            st = run.stats
            hist = st.leaves_history
            key = f"3-{3 + lmax}_{mode}"
            out[key] = {"steps": st.coarse_steps, "regrids": st.regrids,
                        "cell_updates_per_s": st.cell_updates / st.step_seconds, "time_to_solution_s": wall,
                        "leaves_mean": float(np.mean(hist)) if hist else len(run.hier),
                        "l1": l1, "l1_over_paper": l1 / paper[mode][lmax]}
            print(f"[bench] swirl adaptive {key}: {st.coarse_steps} steps, {st.regrids} regrids, "
                  f"{out[key]['cell_updates_per_s']:.3e} cell-updates/s, {wall:.2f} s to solution, leaves "
                  f"{out[key]['leaves_mean']:.0f}, L1 {l1:.4e} ({out[key]['l1_over_paper']:.3f} x Table 3)",
                  file=sys.stderr, flush=True)
            del run
            torch.cuda.empty_cache()
    for mode in ("subcycled", "global"):
        out[f"eoc_{mode}"] = math.log2(out[f"3-4_{mode}"]["l1"] / out[f"3-5_{mode}"]["l1"])
    out["paper_eoc"] = {"subcycled": 2.9705, "global": 2.9703}
    return out


def burgers_runs():
    """Burgers' equation (Sec. 2.2, Sec. 4.4), eq. sinsin01, unlimited.
    Uniform levels 4, 5, 6 (256^2 to 1024^2 cells as 32^2 patches) to
    t = 0.05, before the shock, at CFL 0.5 of |q| <= 1.1, in FP64 and FP32:
    cell-updates/s of the general path and the L1 error against the exact
    implicit solution.  Then the adaptive run of Sec. 4.4: base level 3
    (8x8 patches of 16^2), levels 3-5, a patch refined where a centred
    difference of its averages reaches 15 and coarsened below it, regridded
    every coarse step, to t = 1 (the shock forms at t = 1/(2 pi)); reports
    throughput, leaves and the drift of the conserved sum."""
    import math
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    data, qmax, T = afsynth.burgers_sinsin(), 1.1, 0.05
    out = {}
    for level in (4, 5, 6):
        N, m = 16 << level, 32
        n0 = N // m
        n = math.ceil(T / (0.5 / N / qmax))
        d0 = afsynth.dofs_periodic(data, N, N, nq=4)
        blk = afsynth.periodic_to_blocks(d0, m)
        ex = afsynth.dofs_periodic(afsynth.InitialData(1, lambda x, y: data.exact(x, y, T)), N, N, nq=4)["avg"][0]
        res = {}
        for pname, prec in (("fp64", af.FP64), ("fp32", af.FP32)):
            prob = af.Problem(eq=af.BURGERS, prec=prec, m=m, n0x=n0, n0y=n0, lmax=0, qmax=qmax)
            ctx = af.Context(prob)
            leaves = afsynth.uniform_leaves(n0, n0, 0)
            h = af.Hierarchy(ctx, leaves)
            b0 = af.blocks_to_state(ctx, [{k: blk[k][p] for k in af.KINDS} for p in range(n0 * n0)])
            bufs = [b0, torch.zeros_like(b0)]
            reg = torch.zeros((len(leaves), 4, m, 1), dtype=torch.float64, device="cuda")
            _rot_steps(ctx, h, [b0.clone(), torch.zeros_like(b0)], reg, 2, T / n)  # untimed warm-up
            ms, mask = _event_ms(lambda: _rot_steps(ctx, h, bufs, reg, n, T / n))
            got = af.state_to_blocks(ctx, bufs[mask & 1])
            avg = np.zeros((N, N))
            for p, (_, ix, iy) in enumerate(leaves):
                avg[iy * m:(iy + 1) * m, ix * m:(ix + 1) * m] = got[p]["avg"][0, 2:2 + m, 2:2 + m]
            l1 = float(np.abs(avg - ex).sum()) / N ** 2
            res[pname] = {"steps": n, "ms": ms, "cell_updates_per_s": N * N * n / (ms * 1e-3), "l1": l1}
            print(f"[bench] burgers level {level} ({N}^2) {pname}: {n} steps in {ms:.1f} ms, "
                  f"{res[pname]['cell_updates_per_s']:.3e} cell-updates/s, L1 {l1:.4e}", file=sys.stderr,
                  flush=True)
            del bufs, b0
            torch.cuda.empty_cache()
        out[f"level{level}"] = res
    out["eoc_4_5_fp64"] = math.log2(out["level4"]["fp64"]["l1"] / out["level5"]["fp64"]["l1"])
    out["eoc_5_6_fp64"] = math.log2(out["level5"]["fp64"]["l1"] / out["level6"]["fp64"]["l1"])
    m, n0, lmax, T1 = 16, 8, 2, 1.0
    rule = TagRule(af.TAG_GRADIENT, 0, 15.0, 15.0)
    for pname, prec in (("fp64", af.FP64), ("fp32", af.FP32)):
        prob = af.Problem(eq=af.BURGERS, prec=prec, m=m, n0x=n0, n0y=n0, lmax=lmax, qmax=qmax)

        def block_fn(l, ix, iy, prob=prob):
            dx = prob.dx(l)
            return afsynth.dofs_block(data, m, 2, ix * m * dx, iy * m * dx, dx, dx, 4)

        run = initial_hierarchy(prob, block_fn, rule)
        s0 = float(run.total()[0])
        n = math.ceil(T1 / (0.5 * prob.dx(0) / qmax))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for step in range(n):
            run.coarse_steps(T1 / n, 1)
            if step + 1 < n:
                run.regrid(rule)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s1 = float(run.total()[0])
        st = run.stats
        hist = st.leaves_history
        key = f"adaptive3_5_{pname}"
        out[key] = {"coarse_steps": st.coarse_steps, "regrids": st.regrids,
                    "cell_updates_per_s": st.cell_updates / st.step_seconds, "time_to_solution_s": wall,
                    "leaves_mean": float(np.mean(hist)), "leaves_max": int(max(hist)),
                    "leaves_per_level_final": np.bincount([lv for lv, _, _ in run.hier.leaves()]).tolist(),
                    "sum_drift": abs(s1 - s0), "sum": s0}
        print(f"[bench] burgers adaptive 3-5 {pname}: {st.coarse_steps} coarse steps, {st.regrids} regrids, "
              f"{out[key]['cell_updates_per_s']:.3e} cell-updates/s, {wall:.2f} s to solution, leaves "
              f"{out[key]['leaves_mean']:.0f} (max {out[key]['leaves_max']}), sum drift {abs(s1 - s0):.2e}",
              file=sys.stderr, flush=True)
        del run
        torch.cuda.empty_cache()
    return out


def _rot_steps(ctx, h, bufs, reg, n, dt):
    mask = 0
    for _ in range(n):
        mask = ctx.amr_coarse_step(h, bufs, mask, dt, reg)
    return mask


def cpu_baseline(data, nsteps, dt):
    """The FP64 oracle, single-threaded, on `nsteps` steps of the benchmark
    grid."""
    import afsynth
    import oracle
    d0 = afsynth.dofs_periodic(data, M * N0, M * N0, nq=4)
    t0 = time.perf_counter()
    oracle.run_periodic(0, d0, dt, nsteps, a=1.0, b=0.5)
    el = time.perf_counter() - t0
    return NCELL * nsteps / el, el


_ORACLE_CHILD = """
import sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
z = np.load(sys.argv[2])
d0 = {k: (z[k].item() if z[k].ndim == 0 else z[k]) for k in z.files}
t0 = time.perf_counter()
oracle.run_periodic(0, d0, float(sys.argv[3]), int(sys.argv[4]), a=1.0, b=0.5)
print(time.perf_counter() - t0)
"""


def cpu_baseline_allcore(data, nsteps, dt, nproc):
    """All-core oracle throughput: nproc independent single-threaded oracle
    processes (fresh interpreters that never touch the GPU), each stepping
    its own copy of the benchmark grid; aggregate cell-updates/s over the
    wall time of the slowest."""
    import subprocess
    import tempfile
    import afsynth
    d0 = afsynth.dofs_periodic(data, M * N0, M * N0, nq=4)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "d0.npz")
        np.savez(path, **{k: np.asarray(v) for k, v in d0.items()})
        t0 = time.perf_counter()
        procs = [subprocess.Popen([sys.executable, "-c", _ORACLE_CHILD, ROOT, path, repr(dt), str(nsteps)],
                                  stdout=subprocess.PIPE, text=True) for _ in range(nproc)]
        outs = [p.communicate()[0] for p in procs]
        wall = time.perf_counter() - t0
        if any(p.returncode != 0 for p in procs):
            raise RuntimeError("oracle child failed")
    return nproc * NCELL * nsteps / wall, wall, [float(o.strip()) for o in outs]


def main():
    args = parse()
    if args.peak_probe:
        peak_probe()
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.sweep:
        sweep()
        return
    if args.only:
        runs = {"amr": amr_runs, "rotation": rotation_runs, "swirl": swirl_runs, "burgers": burgers_runs}
        print(json.dumps({args.only: runs[args.only]()}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: --gpus must be 1 (multi-GPU sharding is design-only)"}))
        sys.exit(2)
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    assert torch.cuda.is_available(), "bench needs a GPU"
    data = afsynth.fourier_modes(0)
    dt = T_FINAL / NSTEPS_T
    res = {}
    for name, prec in (("fp32", af.FP32), ("fp64", af.FP64)):
        r = time_path(prec, data, args.steps, args.warmup, dt, args.general_steps)
        res[name] = r
        print(f"[bench] {name}: {args.steps} steps in {r['ms']:.3f} ms; level-advance launch (K={r['K']}, "
              f"{r['NT']} threads) {r['k_ms'] * 1e3:.2f} us; tuned patch step {r['step_us']:.2f} us (tile "
              f"{r['tile']}); general path {r['general_ms_per_step'] * 1e3:.2f} us/step",
              file=sys.stderr, flush=True)
    # accuracy: FP32 vs FP64 (FP64 is parity-tested against the oracle) and
    # both against the exact solution when the run reaches T = 1
    def interior(blocks):
        return np.stack([np.stack([b[k][0, 2:2 + M, 2:2 + M] for k in af.KINDS]) for b in blocks])
    a32, a64 = interior(res["fp32"]["out"]), interior(res["fp64"]["out"])
    linf_32_64 = float(np.abs(a32 - a64).max() / np.abs(a64).max())
    err_exact = None
    if args.steps == NSTEPS_T:
        t = args.steps * dt
        ex = []
        for (l, ix, iy) in afsynth.uniform_leaves(N0, N0, 0):
            dx = 1.0 / (M * N0)
            b = afsynth.dofs_block(afsynth.InitialData(1, lambda x, y: data.exact(x, y, t)), M, 2, ix * M * dx,
                                   iy * M * dx, dx, dx, 4)
            ex.append(b)
        ae = interior(ex)
        err_exact = {"fp32": float(np.abs(a32 - ae).max()), "fp64": float(np.abs(a64 - ae).max())}
    ms32, k32, K32 = res["fp32"]["ms"], res["fp32"]["k_ms"], res["fp32"]["K"]
    ms64, k64 = res["fp64"]["ms"], res["fp64"]["k_ms"]
    ups32 = NCELL * args.steps / (ms32 * 1e-3)
    ups64 = NCELL * args.steps / (ms64 * 1e-3)
    # algorithmic bytes per launch: 8 words (read 4 DOFs, write 4 DOFs) per
    # cell-update, K steps of all 512^2 cells
    bytes32 = 8 * 4 * NCELL * K32
    bytes64 = 8 * 8 * NCELL * res["fp64"]["K"]
    achieved = bytes32 / (k32 * 1e-3) / 1e9
    line = {
        "metric": "cell-updates/s (FP32 vs FP64) of batched AMR AF step; % HBM roofline; L∞ err",
        "value": ups32,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "advection a=1 b=0.5, periodic unit square, one level of 16x16 patches of "
                               "32x32 cells (512^2), 2 ghost layers, seeded 8-mode Fourier data, T=1 "
                               "(1280 steps, CFL 0.4); step = same-level ghost exchange + patch step, "
                               "K steps per launch (af_level_advance, autotuned), launches replayed as one "
                               "HIP graph",
                   "patches": N0 * N0, "patch_cells": M, "steps_per_launch": K32,
                   "threads_per_patch": res["fp32"]["NT"]},
        "eager_ms_per_step": {"fp32": res["fp32"]["eager_ms"] / args.steps,
                              "fp64": res["fp64"]["eager_ms"] / args.steps,
                              "what": "the same launches issued one by one from the library, not replayed"},
        "fp64": {"value": ups64, "ms_per_step": ms64 / args.steps, "kernel_us": k64 * 1e3,
                 "kernel_us_separate_run": res["fp64"]["k_sep"] * 1e3,
                 "steps_per_launch": res["fp64"]["K"], "threads_per_patch": res["fp64"]["NT"],
                 "speedup_fp32_over_fp64": ups32 / ups64,
                 "roofline": {"bound": "hbm", "achieved": bytes64 / (k64 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": bytes64 / (k64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "traffic": PROFILED_TRAFFIC.get(("fp64", res["fp64"]["K"], res["fp64"]["NT"])),
                              "kernel": f"k_level_advance_up<double,32,{res['fp64']['K']},{res['fp64']['NT']}>"}},
        "general_path_us_per_step": {"fp32": res["fp32"]["general_ms_per_step"] * 1e3,
                                     "fp64": res["fp64"]["general_ms_per_step"] * 1e3,
                                     "what": "af_ghost_fill + af_patch_step per step, hipGraph replay"},
        "linf_fp32_vs_fp64_rel": linf_32_64,
        "linf_vs_exact_T1": err_exact,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": PROFILED_TRAFFIC.get(("fp32", K32, res["fp32"]["NT"])),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                     "kernel": f"k_level_advance_up<float,32,{K32},{res['fp32']['NT']}>",
                     "kernel_us": k32 * 1e3, "kernel_us_separate_run": res["fp32"]["k_sep"] * 1e3,
                     "algorithmic_bytes_per_launch": bytes32},
        # the same launch against the vector ALU: the method's flops per
        # cell-update (two time levels of three node stencils, time and face
        # sums, update) over the FP32 peak without packed instructions (256
        # CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s), the
        # ceiling of this build
        "roofline_alu": {"bound": "alu", "achieved": FLOPS_PER_UPDATE[0] * NCELL * K32 / (k32 * 1e-3) / 1e12,
                         "peak": 78.6, "unit": "TFLOP/s",
                         "frac": FLOPS_PER_UPDATE[0] * NCELL * K32 / (k32 * 1e-3) / 1e12 / 78.6,
                         "flops_per_cell_update": FLOPS_PER_UPDATE[0]},
    }
    if not args.no_amr:
        line["amr"] = amr_runs()
        line["rotation"] = rotation_runs()
        line["swirl"] = swirl_runs()
        line["burgers"] = burgers_runs()
    if not args.no_cpu:
        v, el = cpu_baseline(data, args.cpu_steps, dt)
        line["cpu_baseline"] = {"value": v, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
                                "sample": f"{args.cpu_steps} of the 1280 steps on the 512^2 grid "
                                          f"(single-threaded FP64 oracle, {el:.1f} s)"}
        nproc = min(16, len(os.sched_getaffinity(0)))
        va, wa, each = cpu_baseline_allcore(data, args.cpu_steps // 3, dt, nproc)
        line["cpu_baseline_allcore"] = {"value": va, "unit": "cell-updates/s", "cores": nproc, "kind": "oracle",
                                        "sample": f"{nproc} independent oracle processes, {args.cpu_steps // 3} "
                                                  f"steps of the 512^2 grid each, {wa:.1f} s wall "
                                                  f"(slowest process {max(each):.1f} s)"}
        print(f"[bench] oracle: {v:.3e} cell-updates/s on 1 core, {va:.3e} on {nproc} cores", file=sys.stderr,
              flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
