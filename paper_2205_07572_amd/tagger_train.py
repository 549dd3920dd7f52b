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
averages against the exact Fourier solution.
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


def generate(wl: Workload, seeds, horizon=8, every=4, snapshot_stride=2, log=None):
    """Features (unnormalised) and labels from the plain-tagger runs."""
    import torch
    tagger = Tagger()
    xs, ys = [], []
    for seed in seeds:
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


def evaluate(wl: Workload, seeds, tagger=None, horizon=8, every=4):
    """Runs of the held-out seeds; returns a dict per strategy with the mean
    regrid count, wall time, cell updates and L-infinity pressure error."""
    import afsynth
    import torch
    out = {}
    strategies = [("plain_every%d" % every, every, False), ("plain_every%d" % horizon, horizon, False)]
    if tagger is not None:
        strategies.insert(1, ("learned_every%d" % horizon, horizon, True))
    for name, period, learned in strategies:
        rec = {"regrids": [], "wall_s": [], "cell_updates": [], "linf_p": [], "leaves_mean": []}
        for seed in seeds:
            run, data = _new_run(wl, seed)
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
            exact = afsynth.gaussian_pulse_exact(data, wl.alpha)
            err = 0.0
            for b, (l, ix, iy) in zip(run.blocks(), run.hier.leaves()):
                dx = run.prob.dx(l)
                ex = exact.block(run.prob.m, 2, ix * run.prob.m * dx, iy * run.prob.m * dx, dx, dx, wl.T)
                m = run.prob.m
                err = max(err, float(np.abs(b["avg"][0, 2:2 + m, 2:2 + m] - ex["avg"][0, 2:2 + m, 2:2 + m]).max()))
            rec["regrids"].append(run.stats.regrids)
            rec["wall_s"].append(wall)
            rec["cell_updates"].append(run.stats.cell_updates)
            rec["linf_p"].append(err)
            rec["leaves_mean"].append(float(np.mean(leaves)))
        out[name] = {k: float(np.mean(v)) for k, v in rec.items()}
        out[name]["linf_p_max"] = float(np.max(rec["linf_p"]))
    return out


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
