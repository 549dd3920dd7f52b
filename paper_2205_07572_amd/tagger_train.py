"""Training and evaluation of the learned regrid tagger (a project addition,
not part of the paper's method).

Data: adaptive acoustics runs (Gaussian pulse, three levels, plain gradient
tagging every `every` coarse steps).  At each regrid the features of every
leaf are recorded; a shadow copy of the state is advanced `horizon` coarse
steps without regridding and the plain criterion is evaluated on the same
leaves after each of them.  Label: refine if any of those tags is refine,
coarsen if all are coarsen, else keep.

Evaluation: the same runs on held-out seeds with (a) plain tags every
`every` steps, (b) learned tags with the plain fallback every `horizon`
steps, (c) plain tags every `horizon` steps; regrid count, wall time to
solution (regrids included) and the L-infinity error of the pressure
averages against the exact Fourier solution and, optionally, against a
uniform fine-grid run of the same seed (its cell averages restricted to each
leaf's cells).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import ACOUSTICS, FP32, TAG_GRADIENT, Problem, Tagger
from .amr import AMRRun, TagRule, initial_hierarchy


@dataclass
class Workload:
    m: int = 16
    n0: int = 8
    lmax: int = 2
    alpha: float = 200.0
    T: float = 0.5
    cfl: float = 0.4
    prec: int = FP32
    rule: TagRule = None

    def __post_init__(self):
        if self.rule is None:
            self.rule = TagRule(TAG_GRADIENT, 0, 1.0, 0.25)

    def problem(self):
        return Problem(eq=ACOUSTICS, prec=self.prec, m=self.m, n0x=self.n0, n0y=self.n0, lmax=self.lmax, c=1.0)

    def dt0(self, prob):
        n = int(np.ceil(self.T / (self.cfl * prob.dx(0))))
        return self.T / n, n


def _block_fn(prob, data):
    import afsynth

    def fn(l, ix, iy):
        dx = prob.dx(l)
        return afsynth.dofs_block(data, prob.m, 2, ix * prob.m * dx, iy * prob.m * dx, dx, dx, 4)

    return fn


def _new_run(wl: Workload, seed: int):
    import afsynth
    prob = wl.problem()
    data = afsynth.gaussian_pulse(seed, wl.alpha)
    return initial_hierarchy(prob, _block_fn(prob, data), wl.rule), data


def _plain_tags(run: AMRRun, rule: TagRule):
    import torch
    n = len(run.hier)
    t = torch.zeros(n, dtype=torch.int8, device="cuda")
    run.ctx.ghost_fill(run.hier, run.bufs, run.mask, 0, 0)
    run.ctx.regrid_tag(run.hier, run.bufs, run.mask, rule.mode, rule.comp, rule.theta_r, rule.theta_c, t, None)
    return t


def _future_labels(run: AMRRun, dt0, horizon, rule):
    """Plain tags of the current leaves over the next `horizon` coarse steps of
    a shadow copy; returns class labels 0 coarsen, 1 keep, 2 refine."""
    import torch
    bufs = [run.bufs[0].clone(), run.bufs[1].clone()]
    reg = torch.zeros_like(run.reg)
    mask = run.mask
    n = len(run.hier)
    any_ref = torch.zeros(n, dtype=torch.bool, device="cuda")
    all_coarse = torch.ones(n, dtype=torch.bool, device="cuda")
    t = torch.zeros(n, dtype=torch.int8, device="cuda")
    for _ in range(horizon):
        mask = run.ctx.amr_coarse_step(run.hier, bufs, mask, dt0, reg, False)
        run.ctx.ghost_fill(run.hier, bufs, mask, 0, 0)
        run.ctx.regrid_tag(run.hier, bufs, mask, rule.mode, rule.comp, rule.theta_r, rule.theta_c, t, None)
        any_ref |= t == 1
        all_coarse &= t == -1
    lab = torch.ones(n, dtype=torch.int32, device="cuda")
    lab[all_coarse] = 0
    lab[any_ref] = 2
    return lab


def generate(wl: Workload, seeds, horizon=8, every=4, snapshot_stride=2, max_per_seed=None, log=None):
    """Features (unnormalised) and labels from the plain-tagger runs; with
    max_per_seed, a seeded random subset of each run's samples."""
    import torch
    tagger = Tagger()
    xs, ys = [], []
    for seed in seeds:
        n0 = len(xs)
        run, _ = _new_run(wl, seed)
        dt0, nsteps = wl.dt0(run.prob)
        step = 0
        k = 0
        while step + every <= nsteps:
            run.coarse_steps(dt0, every)
            step += every
            run.regrid(wl.rule)
            if k % snapshot_stride == 0 and step + horizon <= nsteps:
                xs.append(tagger.features(run.ctx, run.hier, run.bufs, run.mask))
                ys.append(_future_labels(run, dt0, horizon, wl.rule))
            k += 1
        if max_per_seed is not None:
            xr, yr = torch.cat(xs[n0:]), torch.cat(ys[n0:])
            if len(yr) > max_per_seed:
                g = torch.Generator(device="cpu").manual_seed(1000003 * seed + 17)
                keep = torch.randperm(len(yr), generator=g)[:max_per_seed].cuda()
                xr, yr = xr[keep].contiguous(), yr[keep].contiguous()
            del xs[n0:], ys[n0:]
            xs.append(xr)
            ys.append(yr)
        if log:
            log(f"seed {seed}: {sum(len(y) for y in ys)} samples so far")
    x = torch.cat(xs)
    y = torch.cat(ys)
    return x, y


def normalisation(x):
    """Per-channel mean and inverse standard deviation of features [N][C][16][16]."""
    mean = x.mean(dim=(0, 2, 3))
    inv = 1.0 / x.std(dim=(0, 2, 3)).clamp_min(1e-6)
    return mean, inv


def train(x, y, steps=1500, batch=256, lr=2e-3, seed=0, log=None):
    """Adam on the GPU with the library's own forward/backward kernels.
    Classes are balanced by sampling.  Returns the trained Tagger."""
    import torch
    mean, inv = normalisation(x)
    xn = (x - mean[None, :, None, None]) * inv[None, :, None, None]
    tagger = Tagger()
    rng = np.random.default_rng(seed)
    tagger.set_params(_init_params(tagger.nparams, rng))
    tagger.set_normalization(mean.cpu().numpy(), inv.cpu().numpy())
    tagger.mean, tagger.inv = mean, inv
    ycpu = y.cpu().numpy()
    idx_by_class = [np.nonzero(ycpu == c)[0] for c in range(3)]
    present = [c for c in range(3) if len(idx_by_class[c])]
    losses = []
    for it in range(steps):
        per = batch // len(present)
        sel = np.concatenate([rng.choice(idx_by_class[c], per) for c in present])
        si = torch.from_numpy(sel).cuda()
        loss = tagger.loss_grad(xn[si].contiguous(), y[si].contiguous())
        tagger.adam_step(lr if it < 0.7 * steps else 0.3 * lr)
        if it % 100 == 0:
            losses.append(float(loss.item()))
            if log:
                log(f"step {it}: loss {losses[-1]:.4f}")
    return tagger, losses


def _init_params(n, rng):
    """He-style initialisation of the packed parameters (nin = 13)."""
    p = np.zeros(n, np.float32)
    o = 0
    for cin in (13, 32, 32):
        k = 32 * cin * 9
        p[o:o + k] = rng.standard_normal(k) * np.sqrt(2.0 / (cin * 9))
        o += k + 32
    p[o:o + 96] = rng.standard_normal(96) * np.sqrt(1.0 / 32)
    return p


def accuracy(tagger, x, y):
    """Class accuracy and confusion matrix (rows: label, columns: prediction)
    of the trained network on unnormalised features x."""
    xn = (x - tagger.mean[None, :, None, None]) * tagger.inv[None, :, None, None]
    pred = []
    for i in range(0, len(xn), 4096):
        pred.append(tagger.forward(xn[i:i + 4096].contiguous()).argmax(dim=1))
    import torch
    pred = torch.cat(pred).cpu().numpy()
    yy = y.cpu().numpy()
    conf = np.zeros((3, 3), np.int64)
    for a, b in zip(yy, pred):
        conf[a, b] += 1
    return float((pred == yy).mean()), conf


def pulse_grid_dofs(data, alpha, n, dtype, device="cuda"):
    """Exact DOFs of the pressure of gaussian_pulse on the periodic n x n grid
    at t = 0, as device tensors [n][n] (avg, corner, xedge, yedge): its
    Fourier series evaluated as tensor products (averages with the sinc
    factors of the cell), on `device`."""
    import torch
    import afsynth
    ex = afsynth.gaussian_pulse_exact(data, alpha)
    k = torch.tensor(ex.kx, dtype=torch.float64, device=device)
    P = torch.tensor(ex.phat, dtype=torch.complex128, device=device)  # [a][b]: kx = k[a], ky = k[b]
    h = 1.0 / n
    nodes = torch.arange(n, dtype=torch.float64, device=device) * h
    centres = nodes + 0.5 * h
    sinc = torch.sinc(k * h / 2 / np.pi).to(torch.complex128)

    def f(pos, avg):
        e = torch.exp(1j * torch.outer(pos, k).to(torch.complex128))  # [n][K]
        return e * sinc[None] if avg else e

    def values(xs, ys, avg):
        return torch.real(f(ys, avg) @ P.T @ f(xs, avg).T).to(dtype)  # [y][x]

    return {"avg": values(centres, centres, True), "corner": values(nodes, nodes, False),
            "xedge": values(nodes, centres, False), "yedge": values(centres, nodes, False)}


def uniform_reference(data, wl: Workload, n=4096, m=16, prec=None, log=None):
    """Pressure cell averages [n][n] (device) of the uniform n x n run of
    the same pulse to wl.T (m x m patches, one level, af_level_advance),
    with the time step of the workload's CFL number."""
    import torch
    from . import FP64, Context, Hierarchy
    prec = FP64 if prec is None else prec
    dt_ = torch.float64 if prec == FP64 else torch.float32
    npch = n // m
    prob = Problem(eq=ACOUSTICS, prec=prec, m=m, n0x=npch, n0y=npch, lmax=0, c=1.0)
    ctx = Context(prob)
    hier = Hierarchy(ctx, [(0, ix, iy) for iy in range(npch) for ix in range(npch)])
    g = pulse_grid_dofs(data, wl.alpha, n, dt_)
    st = ctx.new_state(npch * npch)
    idx = torch.arange(-2, m + 3, device="cuda")
    base = torch.arange(npch, device="cuda") * m
    rows = (base[:, None] + idx[None, :]) % n  # [patch row][local row]
    for kk, kind in enumerate(("avg", "corner", "xedge", "yedge")):
        a = g[kind][rows[:, None, :, None], rows[None, :, None, :]]  # [iy][ix][r][c]
        st[kk, 0] = a.reshape(npch * npch, m + 5, m + 5)
    del g
    bufs = [st, torch.zeros_like(st)]
    nsteps = int(np.ceil(wl.T / (wl.cfl * prob.dx(0))))
    dt = wl.T / nsteps
    t0 = time.perf_counter()
    mask = ctx.level_advance(hier, bufs, 0, 0, dt, nsteps)
    torch.cuda.synchronize()
    if log:
        log(f"uniform {n}^2 reference: {nsteps} steps in {time.perf_counter() - t0:.1f} s")
    out = bufs[mask & 1][0, 0, :, 2:2 + m, 2:2 + m].reshape(npch, npch, m, m).permute(0, 2, 1, 3).reshape(n, n)
    return out.to(torch.float64).contiguous()


def _errors(run, wl, data, ref):
    """L-infinity of the leaves' pressure averages against the exact Fourier
    solution and (ref: uniform fine averages [n][n]) against the fine
    averages over each leaf cell."""
    import afsynth
    import torch
    exact = afsynth.gaussian_pulse_exact(data, wl.alpha)
    m = run.prob.m
    pooled = {}
    e_ex = e_ref = 0.0
    for b, (l, ix, iy) in zip(run.blocks(), run.hier.leaves()):
        dx = run.prob.dx(l)
        got = b["avg"][0, 2:2 + m, 2:2 + m]
        ex = exact.block(m, 2, ix * m * dx, iy * m * dx, dx, dx, wl.T)["avg"][0, 2:2 + m, 2:2 + m]
        e_ex = max(e_ex, float(np.abs(got - ex).max()))
        if ref is not None:
            if l not in pooled:
                f = int(round(ref.shape[0] * dx))
                pooled[l] = torch.nn.functional.avg_pool2d(ref[None, None], f)[0, 0].cpu().numpy()
            r = pooled[l][iy * m:(iy + 1) * m, ix * m:(ix + 1) * m]
            e_ref = max(e_ref, float(np.abs(got - r).max()))
    return e_ex, (e_ref if ref is not None else None)


def evaluate(wl: Workload, seeds, tagger=None, horizon=8, every=4, ref_n=None, log=None):
    """Runs of the held-out seeds; returns a dict per strategy with the mean
    regrid count, wall time, cell updates and L-infinity pressure errors
    (against the exact solution; with ref_n also against the uniform ref_n^2
    run of each seed)."""
    import afsynth
    import torch
    out = {}
    strategies = [("plain_every%d" % every, every, False), ("plain_every%d" % horizon, horizon, False)]
    if tagger is not None:
        strategies.insert(1, ("learned_every%d" % horizon, horizon, True))
    recs = {name: {"regrids": [], "wall_s": [], "cell_updates": [], "linf_p": [], "linf_p_ref": [],
                   "leaves_mean": []} for name, _, _ in strategies}
    ref_err = []
    for seed in seeds:
        data = afsynth.gaussian_pulse(seed, wl.alpha)
        ref = uniform_reference(data, wl, ref_n) if ref_n else None
        if ref is not None:
            # the reference's own error, against the exact averages on a 1/16 sample of its rows
            ex = afsynth.gaussian_pulse_exact(data, wl.alpha)
            ys = (np.arange(0, ref_n, 16) + 0.5) / ref_n
            xs = (np.arange(ref_n) + 0.5) / ref_n
            ev = ex.grid_values(xs, ys, wl.T, 1.0 / ref_n, 1.0 / ref_n)[0]
            ref_err.append(float(np.abs(ref[::16].cpu().numpy() - ev).max()))
        for name, period, learned in strategies:
            run, _ = _new_run(wl, seed)
            dt0, nsteps = wl.dt0(run.prob)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step = 0
            leaves = []
            while step < nsteps:
                k = min(period, nsteps - step)
                run.coarse_steps(dt0, k)
                step += k
                leaves.append(len(run.hier))
                if step < nsteps:
                    if learned:
                        plain = _plain_tags(run, wl.rule)
                        tags, _ = tagger.tag(run.ctx, run.hier, run.bufs, run.mask, plain)
                        run.regrid(tags=tags.cpu().numpy())
                    else:
                        run.regrid(wl.rule)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            e_ex, e_ref = _errors(run, wl, data, ref)
            rec = recs[name]
            rec["regrids"].append(run.stats.regrids)
            rec["wall_s"].append(wall)
            rec["cell_updates"].append(run.stats.cell_updates)
            rec["linf_p"].append(e_ex)
            rec["linf_p_ref"].append(e_ref if e_ref is not None else float("nan"))
            rec["leaves_mean"].append(float(np.mean(leaves)))
            del run
        del ref
        torch.cuda.empty_cache()
        if log:
            log(f"seed {seed}: " + ", ".join(f"{n} {recs[n]['regrids'][-1]} regrids L-inf {recs[n]['linf_p'][-1]:.3e}"
                                            for n, _, _ in strategies))
    for name, rec in recs.items():
        out[name] = {k: float(np.mean(v)) for k, v in rec.items()}
        out[name]["linf_p_max"] = float(np.max(rec["linf_p"]))
        if ref_n:
            out[name]["linf_p_ref_max"] = float(np.max(rec["linf_p_ref"]))
        else:
            del out[name]["linf_p_ref"]
    if ref_n:
        out["reference"] = {"n": ref_n, "linf_p_vs_exact_max": float(np.max(ref_err))}
    return out


def config5(train_seeds=range(200), eval_seeds=range(200, 220), steps=2000, horizon=8, every=4,
            max_per_seed=2000, ref_n=4096, log=None):
    """The learned-tagger workload: config-3 runs (Gaussian pulse, three
    levels) with plain tags give the training data; the network is trained
    on the GPU; held-out seeds compare plain tagging every `every` steps,
    learned tagging every `horizon` steps and plain tagging every `horizon`
    steps."""
    import torch
    wl = Workload()
    t0 = time.perf_counter()
    x, y = generate(wl, train_seeds, horizon=horizon, every=every, max_per_seed=max_per_seed, log=log)
    tgen = time.perf_counter() - t0
    counts = np.bincount(y.cpu().numpy(), minlength=3).tolist()
    t0 = time.perf_counter()
    tagger, losses = train(x, y, steps=steps, log=log)
    torch.cuda.synchronize()
    ttrain = time.perf_counter() - t0
    del x, y
    xv, yv = generate(wl, list(eval_seeds)[:2], horizon=horizon, every=every)
    acc, conf = accuracy(tagger, xv, yv)
    del xv, yv
    ev = evaluate(wl, eval_seeds, tagger, horizon=horizon, every=every, ref_n=ref_n, log=log)
    return {"train_seeds": [min(train_seeds), max(train_seeds)], "eval_seeds": [min(eval_seeds), max(eval_seeds)],
            "samples": int(sum(counts)), "class_counts": counts, "max_per_seed": max_per_seed,
            "gen_s": tgen, "train_steps": steps, "train_s": ttrain, "losses": losses,
            "heldout_accuracy": acc, "confusion": conf.tolist(), "eval": ev}


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", type=int, default=12)
    ap.add_argument("--eval-seeds", type=int, default=4)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--T", type=float, default=0.5)
    args = ap.parse_args()
    wl = Workload(T=args.T)
    log = lambda s: print("[tagger]", s, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    x, y = generate(wl, range(args.train_seeds), log=log)
    tgen = time.perf_counter() - t0
    xv, yv = generate(wl, range(200, 200 + max(1, args.eval_seeds // 2)), log=log)
    counts = np.bincount(y.cpu().numpy(), minlength=3).tolist()
    t0 = time.perf_counter()
    tagger, losses = train(x, y, steps=args.steps, log=log)
    ttrain = time.perf_counter() - t0
    acc, conf = accuracy(tagger, xv, yv)
    log(f"held-out accuracy {acc:.3f}, confusion {conf.tolist()}")
    ev = evaluate(wl, range(200, 200 + args.eval_seeds), tagger)
    print(json.dumps({"samples": int(len(y)), "class_counts": counts, "gen_s": tgen, "train_s": ttrain,
                      "losses": losses, "heldout_accuracy": acc, "confusion": conf.tolist(), "eval": ev}), flush=True)


if __name__ == "__main__":
    main()
