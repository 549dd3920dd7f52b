"""Adaptive runs on the GPU: initial hierarchy, subcycled coarse steps with
the conservative fix, periodic regridding (Sec. 3).

Only calls into libaf.so; tags cross to the host once per regrid (the only
device-to-host transfer of the loop), the host computes the new leaf set
(af_hier_regrid), the device transfers the DOFs (af_regrid_apply) and fills
the ghosts.  Coarse steps are launched eagerly by default; hipGraph replay
(captured anew per hierarchy) is optional.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import ACOUSTICS, ADVECTION, FP32, FP64, TAG_GRADIENT, Context, Hierarchy, Problem, blocks_to_state


@dataclass
class TagRule:
    mode: int = TAG_GRADIENT
    comp: int = 0
    theta_r: float = 1.0
    theta_c: float = 0.25


@dataclass
class AMRStats:
    coarse_steps: int = 0
    regrids: int = 0
    cell_updates: int = 0
    step_seconds: float = 0.0      # device time of the coarse steps (events)
    regrid_seconds: float = 0.0    # wall time of the regrids
    leaves_history: list = field(default_factory=list)


class AMRRun:
    """State of one adaptive run: a hierarchy, two state buffers holding the
    levels (per-level buffer mask), FP64 flux registers."""

    def __init__(self, prob: Problem, leaves, block_fn, capacity=None):
        import torch
        self.torch = torch
        self.prob = prob
        self.ctx = Context(prob)
        self.hier = Hierarchy(self.ctx, leaves)
        self.capacity = capacity or max(len(leaves), 64)
        self.block_fn = block_fn  # (level, ix, iy) -> block dict (initial data)
        self.time = 0.0  # time of the synchronised state (time-dependent fields)
        self._alloc(self.capacity)
        self._load_blocks([block_fn(*l) for l in self.hier.leaves()])
        self.stats = AMRStats()

    # ------------------------------------------------------------------ buffers
    def _alloc(self, cap):
        self.capacity = cap
        b0 = self.ctx.new_state(cap)
        self.bufs = [b0, self.torch.zeros_like(b0)]
        self.reg = self.torch.zeros((cap, 4, self.prob.m, self.prob.ncomp), dtype=self.torch.float64,
                                    device="cuda")
        self.mask = 0

    def _load_blocks(self, blocks):
        t = blocks_to_state(self.ctx, blocks, npatch=self.capacity)
        self.bufs[0].copy_(t)
        self.mask = 0
        self.ctx.ghost_fill(self.hier, self.bufs, self.mask, 0, 0)

    def blocks(self):
        """Leaf blocks (host, FP64) in hierarchy order."""
        from . import state_to_blocks
        self.torch.cuda.synchronize()
        n = len(self.hier)
        b = [state_to_blocks(self.ctx, self.bufs[0], n), state_to_blocks(self.ctx, self.bufs[1], n)]
        return [b[(self.mask >> l) & 1][k] for k, (l, _, _) in enumerate(self.hier.leaves())]

    # ------------------------------------------------------------------ steps
    def cell_updates_per_coarse_step(self):
        m2 = self.prob.m ** 2
        return sum(m2 << l for l, _, _ in self.hier.leaves())

    def coarse_steps(self, dt0, n, use_graph=False, global_step=False):
        """n coarse steps of dt0 with subcycling, or with global_step n steps
        of dt0 on every level at once (dt0 then bounded by the finest level's
        CFL)."""
        torch = self.torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        if not use_graph and self.prob.eq in (ADVECTION, ACOUSTICS):
            # constant coefficients (no dependence on t0): all n in one call,
            # one launch fewer per step on the batched path
            self.mask = self.ctx.amr_coarse_steps(self.hier, self.bufs, self.mask, dt0, n, self.reg,
                                                  t0=self.time, global_step=global_step)
            for _ in range(n):
                self.time += dt0
        else:
            for _ in range(n):
                self.mask = self.ctx.amr_coarse_step(self.hier, self.bufs, self.mask, dt0, self.reg, use_graph,
                                                     t0=self.time, global_step=global_step)
                self.time += dt0
        e1.record()
        torch.cuda.synchronize()
        self.stats.step_seconds += e0.elapsed_time(e1) * 1e-3
        self.stats.coarse_steps += n
        per = len(self.hier) * self.prob.m ** 2 if global_step else self.cell_updates_per_coarse_step()
        self.stats.cell_updates += n * per

    def total(self):
        out = self.torch.zeros(self.prob.ncomp, dtype=self.torch.float64, device="cuda")
        self.ctx.reduce_sum(self.hier, self.bufs, self.mask, out)
        return out.cpu().numpy()

    # ------------------------------------------------------------------ regrid
    def tags(self, rule: TagRule):
        torch = self.torch
        n = len(self.hier)
        t = torch.zeros(n, dtype=torch.int8, device="cuda")
        v = torch.zeros(n, dtype=torch.float64, device="cuda")
        self.ctx.ghost_fill(self.hier, self.bufs, self.mask, 0, 0)
        self.ctx.regrid_tag(self.hier, self.bufs, self.mask, rule.mode, rule.comp, rule.theta_r, rule.theta_c, t, v)
        return t.cpu().numpy(), v.cpu().numpy()

    def regrid(self, rule: TagRule = None, tags=None):
        """Tag (or use the given tags), build the new leaf set, transfer the
        DOFs and fill the ghosts.  Returns the tags used.  The transfer reads
        a filled state either way, so that boundary nodes on coarse-fine
        lines hold the finest leaf's values (the fill rule of Sec. 3.1) before
        a coarse leaf hands them to its children."""
        t0 = time.perf_counter()
        if tags is None:
            tags, _ = self.tags(rule)  # fills, then tags
        else:
            self.ctx.ghost_fill(self.hier, self.bufs, self.mask, 0, 0)
        new = self.hier.regrid(tags)
        n = len(new)
        cap = self.capacity
        if n > cap:
            cap = max(n, int(1.5 * cap))
        dst = self.ctx.new_state(cap)
        self.ctx.regrid_apply(self.hier, self.bufs, self.mask, new, dst)
        self.hier = new
        if cap != self.capacity:
            self._alloc(cap)
        self.bufs[0] = dst
        self.bufs[1] = self.torch.zeros_like(dst)
        self.mask = 0
        self.ctx.ghost_fill(self.hier, self.bufs, 0, 0, 0)
        self.torch.cuda.synchronize()
        self.stats.regrids += 1
        self.stats.regrid_seconds += time.perf_counter() - t0
        self.stats.leaves_history.append(n)
        return tags

    def reinit(self):
        """Overwrite every leaf with the initial data (used while building the
        initial hierarchy)."""
        self._load_blocks([self.block_fn(*l) for l in self.hier.leaves()])


def initial_hierarchy(prob: Problem, block_fn, rule: TagRule, passes=None):
    """Start from the uniform level-0 mesh; `passes` times: evaluate the
    initial data, tag, regrid and re-evaluate (the finest level can only be
    reached by one refinement per pass)."""
    leaves = [(0, ix, iy) for iy in range(prob.n0y) for ix in range(prob.n0x)]
    run = AMRRun(prob, leaves, block_fn)
    for _ in range(passes if passes is not None else prob.lmax):
        run.regrid(rule)
        run.reinit()
    run.stats = AMRStats()
    return run
