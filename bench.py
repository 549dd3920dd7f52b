"""Benchmark: the batched adaptive Active Flux step on one MI355X.

Headline workload (config 4): 2D acoustics (p, u, v), c = 1, on the periodic
unit square; a high-frequency wave packet p0 = exp(-50 |x - x0|^2) cos(k.x),
|k| = 80 pi, u = v = 0 (seed 0); 16x16-cell patches with two ghost layers on
8x8 level-0 patches and 4 levels (ratio 2, subcycling, conservative fix);
gradient tagging of p (refine at 8, coarsen below 2), FP32 state and
arithmetic with FP64 flux registers.  One "step" is one coarse step of the
whole hierarchy: one batched launch per even substep start time (4 for 4
levels; each also takes the finest level's second substep) plus the
launches of the conservative fix and vertex copies.  The timed hierarchy is the run's state at
t = T/2 = 0.25 (the initial hierarchy advanced with a regrid every 4 coarse
steps), frozen during the warm-up and the timed steps; cell-updates/s counts
interior leaf cells advanced by their level's step.  FP64 is timed beside
it.  The oracle (single-threaded FP64 C++) runs the first coarse step of the
same workload in a separate process while the GPU is timed; its rate is the
CPU baseline and its result the reference of the FP32 and FP64 L-infinity
errors.

Secondary blocks: config 2 (uniform 512^2 advection, level advance), the full
adaptive runs of configs 3 and 4 to T with regrids (time to solution), and
the rotation, swirl and Burgers runs.

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
# Vector ALU peak of these kernels: 256 CUs x 64 fused multiply-adds per clock
# (FP32 or FP64) x 2 flops x 2.4 GHz = 78.6 TFLOP/s.  The FP32 figure of
# 157.3 TFLOP/s counts packed FP32 instructions, which the library's kernels
# are compiled without.
VALU_PEAK_TFLOPS = 78.6
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


# Config-4 step kernel (k_amr_step, acoustics): algorithmic HBM bytes per leaf
# cell a launch steps (read and write the 4 DOF kinds of 3 components once;
# a fused pair of finest-level substeps makes two cell-updates of them) and
# the operations per cell-update of the orbit-form evaluation
# (af_kernels.hip): 416 node operations (186 additions, 230 multiply-adds) =
# 646 flops, time sums and update about 60 more.
C4_BYTES_PER_CELL = {"fp32": 96, "fp64": 192}
C4_FLOPS_PER_UPDATE = 706
C4_T, C4_EVERY, C4_M, C4_N0, C4_LMAX, C4_THETA = 0.5, 4, 16, 8, 3, (8.0, 2.0)


# HBM bytes per launch of the config-4 step kernel in the timed region (the
# last batched launches of `bench.py --c4-profile`), from rocprofv3
# FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00 KiB (the factors a plain 64 MiB
# device copy gives), valid for the kernel source whose hash is recorded
# (profiles/k_amr_step_config4.md holds the commands).
C4_TRAFFIC = {"source_sha256_16": "50aba14026eab9fa", "fp32": 76885481, "fp64": 147248083}


def _kernel_source_hash(text=None):
    """sha256 prefix of af_kernels.hip with comments and blank space removed
    (the counters depend on the code, not on its comments)."""
    import hashlib
    import re
    if text is None:
        text = open(os.path.join(ROOT, "paper_2205_07572_amd", "csrc", "af_kernels.hip")).read()
    code = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    code = re.sub(r"//[^\n]*", " ", code)
    code = " ".join(code.split())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def c4_traffic(name):
    """Measured HBM bytes per step launch, or None if the kernel source
    changed since the counters were taken."""
    if C4_TRAFFIC["source_sha256_16"] != _kernel_source_hash():
        return None
    return C4_TRAFFIC.get(name)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20, help="timed coarse steps of config 4")
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--c2-steps", type=int, default=NSTEPS_T, help="steps of the config-2 block (T = 1 at 1280)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--general-steps", type=int, default=128)
    p.add_argument("--no-amr", action="store_true", help="skip the adaptive acoustics runs")
    p.add_argument("--sweep", action="store_true",
                   help="roofline sweep: uniform grids up to 4096^2 (HBM resident); one JSON line per case")
    p.add_argument("--copy-probe", action="store_true",
                   help="only run a plain 64 MiB device copy 20 times (HBM counter calibration)")
    p.add_argument("--peak-probe", action="store_true",
                   help="only measure the device's copy bandwidth and vector FMA rate (one JSON line)")
    p.add_argument("--config5", action="store_true",
                   help="the learned-tagger workload instead of the benchmark line: train on config-3 runs, "
                        "evaluate held-out seeds against plain tagging and a uniform fine run (minutes)")
    p.add_argument("--c5-train-seeds", type=int, default=200)
    p.add_argument("--c5-eval-seeds", type=int, default=20)
    p.add_argument("--c5-ref-n", type=int, default=4096)
    p.add_argument("--c5-steps", type=int, default=2000)
    p.add_argument("--c4-profile", choices=["fp32", "fp64"],
                   help="only the config-4 timed step in that precision (for a profiler run)")
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
# instructions are disabled for every kernel of the library, so FP32 kernels
# can reach at most half of the FP32 figure.
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


class HipEvents:
    """Raw HIP events (timing enabled) through the HIP runtime torch has
    loaded, for the library's timed coarse step."""

    def __init__(self, n):
        import ctypes
        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(n):
            e = ctypes.c_void_p()
            assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
            self.ev.append(e.value)

    def handles(self, first, count):
        return self.ev[first:first + count]

    def ms(self, a, b):
        t = self.ct.c_float()
        assert self.hip.hipEventElapsedTime(self.ct.byref(t), self.ev[a], self.ev[b]) == 0
        return float(t.value)

    def __del__(self):
        for e in getattr(self, "ev", []):
            self.hip.hipEventDestroy(e)


def c4_problem(prec):
    import paper_2205_07572_amd as af
    return af.Problem(eq=af.ACOUSTICS, prec=prec, m=C4_M, n0x=C4_N0, n0y=C4_N0, lmax=C4_LMAX, c=1.0)


def c4_initial(prec):
    """The config-4 run's initial hierarchy (exact data, lmax passes of
    gradient tagging and refinement) and its coarse time step."""
    import math
    import afsynth
    import paper_2205_07572_amd as af
    from paper_2205_07572_amd.amr import TagRule, initial_hierarchy
    prob = c4_problem(prec)
    data = afsynth.wave_packet(0)

    def block_fn(l, ix, iy):
        dx = prob.dx(l)
        return afsynth.dofs_block(data, C4_M, 2, ix * C4_M * dx, iy * C4_M * dx, dx, dx, 4)

    rule = TagRule(af.TAG_GRADIENT, 0, *C4_THETA)
    run = initial_hierarchy(prob, block_fn, rule)
    n = math.ceil(C4_T / (0.4 * prob.dx(0)))
    return run, rule, C4_T / n, n


def c4_headline(prec, steps, warmup):
    """The timed config-4 step: the run advanced to t = T/2 with a regrid
    every 4 coarse steps, then `warmup` coarse steps and two timed regions of
    `steps` coarse steps each on that hierarchy.  The first is `steps` plain
    batched coarse steps in one call between two events (the throughput).  The second
    records HIP events around every batched step launch on the stream it
    runs on (the dominant kernel's launch times); those event records cost
    about a tenth of the step time, so they stay out of the first region."""
    import torch
    import paper_2205_07572_amd as af
    run, rule, dt0, n = c4_initial(prec)
    half = n // 2
    step = 0
    while step < half:
        k = min(C4_EVERY, half - step)
        run.coarse_steps(dt0, k)
        step += k
        if step < half:
            run.regrid(rule)
    leaves = run.hier.leaves()
    per_step = run.cell_updates_per_coarse_step()
    ctx, h = run.ctx, run.hier
    for _ in range(warmup):
        run.mask = ctx.amr_coarse_step(h, run.bufs, run.mask, dt0, run.reg, t0=run.time)
        run.time += dt0
    # region 1: throughput
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record()
    # the `steps` coarse steps in one call: the state between them is not
    # read, so each step's last fix shares a launch with the next step's
    # vertex copies (af_amr_coarse_steps; the same result as single steps)
    run.mask = ctx.amr_coarse_steps(h, run.bufs, run.mask, dt0, steps, run.reg, t0=run.time)
    for _ in range(steps):
        run.time += dt0
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    # region 2: launch times of the batched step kernel
    nmax = 1 << C4_LMAX  # batched step launches per coarse step, at most
    ev = HipEvents(2 * nmax * steps)
    cells = []
    torch.cuda.synchronize()
    e0.record()
    for k in range(steps):
        run.mask, nl, c = ctx.amr_coarse_step_timed(h, run.bufs, run.mask, dt0, run.reg,
                                                    ev.handles(2 * nmax * k, 2 * nmax), t0=run.time)
        run.time += dt0
        cells.append((nl, c))
    e1.record()
    torch.cuda.synchronize()
    ms_timed = e0.elapsed_time(e1)
    launch_ms, launch_cells = [], []
    for k, (nl, c) in enumerate(cells):
        for j in range(nl):
            launch_ms.append(ev.ms(2 * nmax * k + 2 * j, 2 * nmax * k + 2 * j + 1))
            launch_cells.append(float(c[j]))
    counts = np.bincount([l for l, _, _ in leaves], minlength=C4_LMAX + 1).tolist()
    # leaf cells each launch reads and writes once: the levels that start a
    # step at its time point tau; with fused pairs (finest level F >= 2,
    # m = 16) the launches are the even tau and level F takes two substeps
    F = max(l for l, _, _ in leaves)
    fused = ctx.fused_pairs and F >= 2 and C4_M in (8, 16)
    leaf_cells = []
    for k, (nl, _) in enumerate(cells):
        for j in range(nl):
            tau = 2 * j if fused else j
            l0 = 0 if tau == 0 else F - ((tau & -tau).bit_length() - 1)
            leaf_cells.append(float(C4_M * C4_M * sum(counts[l0:F + 1])))
            upd = leaf_cells[-1] + (C4_M * C4_M * counts[F] if fused else 0)
            assert upd == launch_cells[len(leaf_cells) - 1], (upd, launch_cells[len(leaf_cells) - 1])
    return dict(ms=ms, ms_timed=ms_timed, wall_s=t_wall, per_step=per_step, leaves=len(leaves), per_level=counts,
                launch_ms=np.array(launch_ms), launch_cells=np.array(launch_cells),
                launch_leaf_cells=np.array(leaf_cells), fused_pairs=fused, dt0=dt0, t_start=half * dt0)


_C4_ORACLE_CHILD = """
import sys, time, json
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
z = np.load(sys.argv[2])
leaves = [tuple(int(v) for v in l) for l in z["leaves"]]
o = oracle.Hier(1, int(z["m"]), int(z["n0"]), int(z["n0"]), int(z["lmax"]), c=1.0)
o.set_leaves(leaves)
for k in range(len(leaves)):
    o.set_block(k, {kind: z[kind][k] for kind in oracle.KINDS})
t0 = time.perf_counter()
o.coarse_step(float(z["dt0"]))
el = time.perf_counter() - t0
if len(sys.argv) > 4 and sys.argv[4] == "time-only":
    np.savez(sys.argv[3], seconds=el)
else:
    out = {kind: np.stack([o.get_block(k)[kind] for k in range(len(leaves))]) for kind in oracle.KINDS}
    np.savez(sys.argv[3], seconds=el, **out)
"""


def c4_oracle_start(tmp):
    """Starts the oracle on the first coarse step of config 4 (FP64, one
    thread, a fresh interpreter that never touches the GPU) from the GPU's
    FP64 initial hierarchy; returns what c4_oracle_finish needs."""
    import subprocess
    import paper_2205_07572_amd as af
    run, _, dt0, _ = c4_initial(af.FP64)
    leaves = run.hier.leaves()
    blocks = run.blocks()
    path = os.path.join(tmp, "c4_init.npz")
    np.savez(path, leaves=np.array(leaves, np.int32), m=C4_M, n0=C4_N0, lmax=C4_LMAX, dt0=dt0,
             **{k: np.stack([b[k] for b in blocks]) for k in ("avg", "corner", "xedge", "yedge")})
    out = os.path.join(tmp, "c4_oracle.npz")
    proc = subprocess.Popen([sys.executable, "-c", _C4_ORACLE_CHILD, ROOT, path, out])
    cu = run.cell_updates_per_coarse_step()
    del run
    return dict(proc=proc, out=out, leaves=leaves, blocks=blocks, dt0=dt0, cell_updates=cu)


def c4_gpu_first_step(job, prec):
    """The same first coarse step on the GPU (from the same FP64 blocks,
    rounded to FP32 for the FP32 path)."""
    import paper_2205_07572_amd as af
    from paper_2205_07572_amd.amr import AMRRun
    by_leaf = {lf: b for lf, b in zip(job["leaves"], job["blocks"])}
    run = AMRRun(c4_problem(prec), job["leaves"], lambda l, ix, iy: by_leaf[(l, ix, iy)])
    run.coarse_steps(job["dt0"], 1)
    return run.blocks()


def c4_oracle_finish(job, gpu):
    """Waits for the oracle; L-infinity of each GPU result against it over
    the interior averages and closed-square nodes of every leaf, relative to
    the state's largest value."""
    if job["proc"].wait() != 0:
        raise RuntimeError("oracle child failed")
    z = np.load(job["out"])
    m = C4_M
    sl = {"avg": (slice(2, 2 + m), slice(2, 2 + m)), "corner": (slice(2, 3 + m), slice(2, 3 + m)),
          "xedge": (slice(2, 2 + m), slice(2, 3 + m)), "yedge": (slice(2, 3 + m), slice(2, 2 + m))}
    scale = max(float(np.abs(z[k][(slice(None), slice(None)) + sl[k]]).max()) for k in sl)
    errs = {}
    for name, blocks in gpu.items():
        e_avg = max(float(np.abs(b["avg"][(slice(None),) + sl["avg"]] - z["avg"][i][(slice(None),) + sl["avg"]]).max())
                    for i, b in enumerate(blocks))
        e_pt = max(float(np.abs(b[k][(slice(None),) + sl[k]] - z[k][i][(slice(None),) + sl[k]]).max())
                   for i, b in enumerate(blocks) for k in ("corner", "xedge", "yedge"))
        errs[name] = {"averages": e_avg / scale, "point_values": e_pt / scale}
    return float(z["seconds"]), errs


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
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: --gpus must be 1 (multi-GPU sharding is design-only)"}))
        sys.exit(2)
    if args.config5:
        from paper_2205_07572_amd import tagger_train as tt
        log = lambda s: print("[config5]", s, file=sys.stderr, flush=True)  # noqa: E731
        r = tt.config5(train_seeds=range(args.c5_train_seeds), eval_seeds=range(200, 200 + args.c5_eval_seeds),
                       steps=args.c5_steps, ref_n=args.c5_ref_n or None, log=log)
        print(json.dumps({"config5": r}), flush=True)
        return
    if args.c4_profile:
        import paper_2205_07572_amd as af
        r = c4_headline(af.FP32 if args.c4_profile == "fp32" else af.FP64, args.steps, args.warmup)
        print(json.dumps({"c4_profile": args.c4_profile, "steps": args.steps, "launches": len(r["launch_ms"]),
                          "launch_us_avg": 1e3 * float(np.mean(r["launch_ms"])),
                          "launch_cells_avg": float(np.mean(r["launch_cells"])),
                          "kernel_source_sha256_16": _kernel_source_hash()}), flush=True)
        return
    if args.only:
        runs = {"amr": amr_runs, "rotation": rotation_runs, "swirl": swirl_runs, "burgers": burgers_runs}
        print(json.dumps({args.only: runs[args.only]()}), flush=True)
        return
    import tempfile
    import torch
    import afsynth
    import paper_2205_07572_amd as af
    assert torch.cuda.is_available(), "bench needs a GPU"
    tmp = tempfile.TemporaryDirectory()
    job = None if args.no_cpu else c4_oracle_start(tmp.name)

    # ---- headline: config 4, FP32 and FP64
    c4 = {}
    for name, prec in (("fp32", af.FP32), ("fp64", af.FP64)):
        r = c4_headline(prec, args.steps, args.warmup)
        c4[name] = r
        us = np.sum(r["launch_ms"]) * 1e3
        print(f"[bench] config4 {name}: {r['leaves']} leaves {r['per_level']}, {args.steps} coarse steps in "
              f"{r['ms']:.3f} ms ({1e3 * r['ms'] / args.steps:.1f} us each), "
              f"{r['per_step'] * args.steps / (r['ms'] * 1e-3):.3e} cell-updates/s; batched step launches "
              f"{len(r['launch_ms'])}, {us / len(r['launch_ms']):.2f} us average", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    r32, r64 = c4["fp32"], c4["fp64"]
    ups32 = r32["per_step"] * args.steps / (r32["ms"] * 1e-3)
    ups64 = r64["per_step"] * args.steps / (r64["ms"] * 1e-3)

    def roofline(r, name):
        """The dominant kernel against the roof its arithmetic intensity
        meets: HBM bytes = the leaf DOFs a launch reads and writes once,
        flops = the orbit-form operations of every cell-update it makes."""
        bytes_ = C4_BYTES_PER_CELL[name] * float(np.sum(r["launch_leaf_cells"]))
        flops = C4_FLOPS_PER_UPDATE * float(np.sum(r["launch_cells"]))
        secs = float(np.sum(r["launch_ms"])) * 1e-3
        gbs, tfl = bytes_ / secs / 1e9, flops / secs / 1e12
        intensity = flops / bytes_
        alu_bound = intensity * HBM_PEAK_GBS * 1e-3 > VALU_PEAK_TFLOPS
        hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
        alu = {"bound": "alu", "achieved": tfl, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": tfl / VALU_PEAK_TFLOPS}
        out = dict(alu if alu_bound else hbm)
        out.update({"traffic": c4_traffic(name),
                    "kernel": f"k_amr_step<{'float' if name == 'fp32' else 'double'},1,16,18,pair>",
                    "launches": int(len(r["launch_ms"])),
                    "kernel_us_avg": 1e3 * float(np.mean(r["launch_ms"])),
                    "algorithmic_bytes_per_launch_avg": bytes_ / len(r["launch_ms"]),
                    "algorithmic_flops_per_launch_avg": flops / len(r["launch_ms"]),
                    "flops_per_byte": intensity,
                    "other_roof": alu if not alu_bound else hbm,
                    "fused_pairs": r["fused_pairs"],
                    "ms_per_step_of_region": r["ms_timed"] / args.steps,
                    "what": "dominant kernel: the batched step launches of a second timed region of the same "
                            "number of coarse steps, HIP events around each on its stream; bytes = bytes per leaf cell (each DOF read and written "
                            "once) x leaf cells of the levels stepping at the launch's time point; flops = "
                            "operations per cell-update x cell-updates (the finest level's fused pair counts "
                            "twice); bound = the lower roof at that intensity (FP32 vector peak without packed "
                            "FP32 instructions)"})
        return out

    def step_roofline(r, name, ups):
        bytes_step = C4_BYTES_PER_CELL[name] * float(np.sum(r["launch_leaf_cells"])) / args.steps
        achieved = bytes_step / (r["ms"] / args.steps * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "alu_tflops": C4_FLOPS_PER_UPDATE * ups / 1e12,
                "alu_frac": C4_FLOPS_PER_UPDATE * ups / 1e12 / VALU_PEAK_TFLOPS,
                "what": "whole coarse step (all launches and the gaps between them): leaf bytes of the step "
                        "launches / ms_per_step, and operations x cell-updates / ms_per_step"}

    line = {
        "metric": "cell-updates/s (FP32 vs FP64) of batched AMR AF step; % HBM roofline; L∞ err",
        "value": ups32,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config 4: acoustics c=1 on the periodic unit square, wave packet "
                               "exp(-50|x-x0|^2) cos(k.x), |k|=80 pi, seed 0; 16x16-cell patches, 8x8 level-0 "
                               "patches, 4 levels (subcycling, conservative fix), gradient tags refine 8 / "
                               "coarsen 2; step = one coarse step of the hierarchy reached at t=T/2=0.25 "
                               "(regrid every 4 coarse steps), FP32 bulk, FP64 flux registers",
                   "leaves": r32["leaves"], "leaves_per_level": r32["per_level"],
                   "cell_updates_per_step": r32["per_step"], "t_start": r32["t_start"], "dt0": r32["dt0"]},
        "roofline": roofline(r32, "fp32"),
        "roofline_step": step_roofline(r32, "fp32", ups32),
        "fp64": {"value": ups64, "ms_per_step": r64["ms"] / args.steps, "leaves": r64["leaves"],
                 "cell_updates_per_step": r64["per_step"], "speedup_fp32_over_fp64": ups32 / ups64,
                 "roofline": roofline(r64, "fp64"), "roofline_step": step_roofline(r64, "fp64", ups64)},
    }
    del c4

    # ---- the oracle's first coarse step: CPU baseline and L-infinity errors
    if job is not None:
        gpu = {"fp32": c4_gpu_first_step(job, af.FP32), "fp64": c4_gpu_first_step(job, af.FP64)}
        secs, errs = c4_oracle_finish(job, gpu)
        line["linf_vs_oracle"] = dict(errs, what="first coarse step of config 4 from the initial hierarchy "
                                                 f"({len(job['leaves'])} leaves), relative to the state's largest "
                                                 "value; the FP32 run starts from the same data rounded to FP32")
        line["cpu_baseline"] = {"value": job["cell_updates"] / secs, "unit": "cell-updates/s", "cores": 1,
                                "kind": "oracle", "cpu": _cpu_model(),
                                "sample": f"the first coarse step of config 4 ({len(job['leaves'])} leaves, "
                                          f"{job['cell_updates']} cell-updates, {secs:.1f} s), single-threaded "
                                          "FP64 oracle in its own process, run while the GPU was timed"}
        print(f"[bench] oracle: config-4 first coarse step {secs:.1f} s, "
              f"{job['cell_updates'] / secs:.3e} cell-updates/s; L-inf vs oracle {errs}", file=sys.stderr,
              flush=True)
        del gpu

    # ---- config 2: uniform advection through the level advance
    data = afsynth.fourier_modes(0)
    dt = T_FINAL / NSTEPS_T
    res = {}
    for name, prec in (("fp32", af.FP32), ("fp64", af.FP64)):
        r = time_path(prec, data, args.c2_steps, 20, dt, args.general_steps)
        res[name] = r
        print(f"[bench] config2 {name}: {args.c2_steps} steps in {r['ms']:.3f} ms; level-advance launch "
              f"(K={r['K']}, {r['NT']} threads) {r['k_ms'] * 1e3:.2f} us", file=sys.stderr, flush=True)
    line["config2"] = config2_block(res, args.c2_steps, dt)
    del res

    if not args.no_amr:
        line["amr_runs"] = amr_runs()
        line["rotation"] = rotation_runs()
        line["swirl"] = swirl_runs()
        line["burgers"] = burgers_runs()
    if job is not None:
        # all host cores: independent oracle processes, each the same first
        # coarse step, after the GPU work (so that they do not compete with
        # its launches)
        nproc = min(16, len(os.sched_getaffinity(0)))
        wall, each = c4_oracle_allcore(job, tmp.name, nproc)
        line["cpu_baseline_allcore"] = {"value": nproc * job["cell_updates"] / wall, "unit": "cell-updates/s",
                                        "cores": nproc, "kind": "oracle", "cpu": _cpu_model(),
                                        "sample": f"{nproc} independent oracle processes, each the first coarse "
                                                  f"step of config 4, {wall:.1f} s wall (slowest {max(each):.1f} s)"}
        print(f"[bench] oracle on {nproc} cores: {nproc * job['cell_updates'] / wall:.3e} cell-updates/s",
              file=sys.stderr, flush=True)
    tmp.cleanup()
    print(json.dumps(line), flush=True)


def c4_oracle_allcore(job, tmp, nproc):
    import subprocess
    path = os.path.join(tmp, "c4_init.npz")
    outs = [os.path.join(tmp, f"c4_oracle_{k}.npz") for k in range(nproc)]
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, "-c", _C4_ORACLE_CHILD, ROOT, path, o, "time-only"]) for o in outs]
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("oracle child failed")
    wall = time.perf_counter() - t0
    return wall, [float(np.load(o)["seconds"]) for o in outs]


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def config2_block(res, steps, dt):
    """Config 2 (512^2 uniform advection, af_level_advance with K steps per
    launch, replayed as a HIP graph): throughput, the roofline of the timed
    region itself (algorithmic bytes per step over ms per step) and of its
    launches, and the measured HBM traffic of a launch."""
    import afsynth
    import paper_2205_07572_amd as af
    out = {"workload": "advection a=1 b=0.5, periodic unit square, 16x16 patches of 32x32 cells (512^2), "
                       "seeded 8-mode Fourier data, CFL 0.4, T=1 in 1280 steps"}

    def interior(blocks):
        return np.stack([np.stack([b[k][0, 2:2 + M, 2:2 + M] for k in af.KINDS]) for b in blocks])

    a32, a64 = interior(res["fp32"]["out"]), interior(res["fp64"]["out"])
    out["linf_fp32_vs_fp64_rel"] = float(np.abs(a32 - a64).max() / np.abs(a64).max())
    for name, wb in (("fp32", 4), ("fp64", 8)):
        r = res[name]
        ms_step = r["ms"] / steps
        bytes_step = 8 * wb * NCELL
        traffic = PROFILED_TRAFFIC.get((name, r["K"], r["NT"]))
        out[name] = {"cell_updates_per_s": NCELL / (ms_step * 1e-3), "ms_per_step": ms_step,
                     "steps_per_launch": r["K"], "threads_per_patch": r["NT"], "kernel_us": r["k_ms"] * 1e3,
                     "effective_bandwidth": {"achieved": bytes_step / (ms_step * 1e-3) / 1e9, "unit": "GB/s",
                                             "algorithmic_frac_of_hbm_peak":
                                                 bytes_step / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                             "what": "algorithmic bytes (8 words per cell-update) / ms per step, "
                                                     "graph replay of the whole run; a launch keeps K steps on "
                                                     "chip, so this effective rate is no HBM fraction and can "
                                                     "exceed the peak (traffic_frac is the counted one)"},
                     "traffic_per_launch": traffic,
                     "traffic_frac": (traffic / (r["k_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "eager_ms_per_step": r["eager_ms"] / steps,
                     "general_path_us_per_step": r["general_ms_per_step"] * 1e3}
    out["speedup_fp32_over_fp64"] = out["fp32"]["cell_updates_per_s"] / out["fp64"]["cell_updates_per_s"]
    if steps == NSTEPS_T:
        t = steps * dt
        ex = []
        for (l, ix, iy) in afsynth.uniform_leaves(N0, N0, 0):
            dx = 1.0 / (M * N0)
            ex.append(afsynth.dofs_block(afsynth.InitialData(1, lambda x, y: afsynth.fourier_modes(0).exact(x, y, t)),
                                         M, 2, ix * M * dx, iy * M * dx, dx, dx, 4))
        ae = interior(ex)
        out["linf_vs_exact_T1"] = {"fp32": float(np.abs(a32 - ae).max()), "fp64": float(np.abs(a64 - ae).max())}
    return out


if __name__ == "__main__":
    main()
