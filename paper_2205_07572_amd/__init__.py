"""MI355X Active Flux patch-step library (Python side).

A thin layer over libaf.so (include/af.h): it allocates state buffers as
torch tensors on the GPU, marshals arguments, and passes torch's current
stream.  All arithmetic of the method runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import AFError, check

ADVECTION, ACOUSTICS, ROTATION, SWIRL, BURGERS = 0, 1, 2, 3, 4
STEP_GRAPH, STEP_GLOBAL = 1, 2
FP64, FP32 = 0, 1
KINDS = ("avg", "corner", "xedge", "yedge")
REGION_INTERIOR, REGION_LAYER1 = 0, 1
TAG_GRADIENT, TAG_MAXMIN = 0, 1


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class Problem:
    eq: int = ADVECTION
    prec: int = FP64
    m: int = 16
    n0x: int = 1
    n0y: int = 1
    lmax: int = 0
    x0: float = 0.0
    y0: float = 0.0
    lx: float = 1.0
    ly: float = 1.0
    a: float = 1.0
    b: float = 0.5
    c: float = 1.0
    omega: float = 0.0   # ROTATION: a = -omega (y - yc), b = omega (x - xc)
    xc: float = 0.0
    yc: float = 0.0
    qmax: float = 0.0    # BURGERS: bound on |q| over the run (CFL check)

    @property
    def ncomp(self):
        return 3 if self.eq == ACOUSTICS else 1

    def dx(self, level):
        return self.lx / (self.n0x * self.m) / 2 ** level

    def dy(self, level):
        return self.ly / (self.n0y * self.m) / 2 ** level


class Context:
    def __init__(self, prob: Problem):
        self.prob = prob
        L = _lib.load()
        cp = _lib.af_problem(prob.eq, prob.prec, prob.m, prob.n0x, prob.n0y, prob.lmax, prob.x0, prob.y0,
                             prob.lx, prob.ly, prob.a, prob.b, prob.c, prob.omega, prob.xc, prob.yc,
                             prob.qmax)
        h = ctypes.c_void_p()
        check(L.af_ctx_create(ctypes.byref(cp), ctypes.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _lib.load().af_ctx_destroy(self.h)
                self.h = None
        except Exception:  # interpreter shutdown
            pass

    @property
    def tile(self):
        return _lib.load().af_ctx_get_tile(self.h)

    @tile.setter
    def tile(self, ty):
        check(_lib.load().af_ctx_set_tile(self.h, int(ty)))

    @property
    def fused_pairs(self):
        """af_ctx_get_fused_pairs: the batched coarse step fuses each pair of
        finest-level substeps into one launch (bit-identical results)."""
        return bool(_lib.load().af_ctx_get_fused_pairs(self.h))

    @fused_pairs.setter
    def fused_pairs(self, on):
        check(_lib.load().af_ctx_set_fused_pairs(self.h, int(bool(on))))

    def advance_shapes(self):
        """(K, threads) pairs of the level-advance kernel for this problem."""
        L = _lib.load()
        n = L.af_ctx_advance_shapes(self.h, None, None, 0)
        ks = np.zeros(max(n, 1), np.int32)
        nts = np.zeros(max(n, 1), np.int32)
        L.af_ctx_advance_shapes(self.h, ks.ctypes.data_as(ctypes.c_void_p), nts.ctypes.data_as(ctypes.c_void_p), n)
        return [(int(k), int(t)) for k, t in zip(ks[:n], nts[:n])]

    def advance_shapes_upwind(self):
        """The (K, threads) pairs of advance_shapes() that only the upwind
        one-pass kernel runs (others fall back to the default shape)."""
        L = _lib.load()
        n = L.af_ctx_advance_shapes_upwind(self.h, None, None, 0)
        ks = np.zeros(max(n, 1), np.int32)
        nts = np.zeros(max(n, 1), np.int32)
        L.af_ctx_advance_shapes_upwind(self.h, ks.ctypes.data_as(ctypes.c_void_p),
                                       nts.ctypes.data_as(ctypes.c_void_p), n)
        return [(int(k), int(t)) for k, t in zip(ks[:n], nts[:n])]

    def set_advance_shape(self, k, nt):
        check(_lib.load().af_ctx_set_advance_shape(self.h, int(k), int(nt)))

    @property
    def advance_shape(self):
        k, nt = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().af_ctx_get_advance_shape(self.h, ctypes.byref(k), ctypes.byref(nt)))
        return k.value, nt.value

    # ----------------------------------------------------------------- state
    def new_state(self, npatch, pitch=None):
        """Zeroed state tensor [4][ncomp][npatch][m+5][pitch] on the GPU."""
        torch = _torch()
        pitch = pitch or (self.prob.m + 5)
        dt = torch.float32 if self.prob.prec == FP32 else torch.float64
        return torch.zeros((4, self.prob.ncomp, npatch, self.prob.m + 5, pitch), dtype=dt, device="cuda")

    @staticmethod
    def cstate(t):
        s = _lib.af_state()
        for k in range(4):
            s.dof[k] = t[k].data_ptr()
        s.npatch = t.shape[2]
        s.pitch = t.shape[4]
        return s

    # ----------------------------------------------------------------- calls
    def patch_step(self, tin, tout, first, count, level, dt, region=REGION_INTERIOR, flux_reg=None,
                   side_mask=None, leaf_xy=None, t=0.0):
        """leaf_xy: device (ix, iy) table of the patches (Hierarchy.leaf_xy_ptr()
        or an int32 tensor [npatch][2]); needed for ROTATION and SWIRL.  t: time
        at the start of the step (SWIRL)."""
        sin, sout = self.cstate(tin), self.cstate(tout)
        sm = ctypes.c_void_p(side_mask) if isinstance(side_mask, int) else _ptr(side_mask)
        xy = ctypes.c_void_p(leaf_xy) if isinstance(leaf_xy, int) else _ptr(leaf_xy)
        check(_lib.load().af_patch_step(self.h, ctypes.byref(sin), ctypes.byref(sout), int(first), int(count),
                                        int(level), float(dt), float(t), int(region), _ptr(flux_reg), sm, xy,
                                        _stream()))

    def _pair(self, bufs):
        arr = (_lib.af_state * 2)()
        arr[0] = self.cstate(bufs[0])
        arr[1] = self.cstate(bufs[1] if len(bufs) > 1 else bufs[0])
        return arr

    def ghost_fill(self, hier, bufs, mask=0, tmin=0, smin=0):
        check(_lib.load().af_ghost_fill(self.h, hier.h, self._pair(bufs), int(mask), int(tmin), int(smin),
                                        _stream()))

    def flux_correct(self, hier, bufs, mask, level, flux_reg):
        check(_lib.load().af_flux_correct(self.h, hier.h, self._pair(bufs), int(mask), int(level),
                                          _ptr(flux_reg), _stream()))

    def regrid_tag(self, hier, bufs, mask, mode, comp, theta_r, theta_c, tags, values=None):
        check(_lib.load().af_regrid_tag(self.h, hier.h, self._pair(bufs), int(mask), int(mode), int(comp),
                                        float(theta_r), float(theta_c), _ptr(tags), _ptr(values), _stream()))

    def regrid_apply(self, old, bufs, mask, new, dst):
        d = self.cstate(dst)
        check(_lib.load().af_regrid_apply(self.h, old.h, self._pair(bufs), int(mask), new.h, ctypes.byref(d),
                                          _stream()))

    def reduce_sum(self, hier, bufs, mask, out):
        check(_lib.load().af_reduce_sum(self.h, hier.h, self._pair(bufs), int(mask), _ptr(out), _stream()))

    def reduce_sum_noalloc(self, hier, bufs, mask, out):
        """af_reduce_sum_noalloc: the same sums with the library's static
        scratch (no device allocation; the hierarchy must be on the device)."""
        check(_lib.load().af_reduce_sum_noalloc(self.h, hier.h, self._pair(bufs), int(mask), _ptr(out),
                                                _stream()))

    def level_advance(self, hier, bufs, mask, level, dt, nsteps):
        mk = ctypes.c_uint32(mask)
        check(_lib.load().af_level_advance(self.h, hier.h, self._pair(bufs), ctypes.byref(mk), int(level),
                                           float(dt), int(nsteps), _stream()))
        return mk.value

    def autotune(self, hier, bufs, level, dt, reps=20):
        """Time every kernel shape and keep the fastest (steps the data in bufs).
        Returns (best patch-step us, best level-advance us per step or -1)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        check(_lib.load().af_autotune(self.h, hier.h, self._pair(bufs), int(level), float(dt), int(reps),
                                      ctypes.byref(a), ctypes.byref(b), _stream()))
        return a.value, b.value

    def amr_coarse_step(self, hier, bufs, mask, dt0, flux_reg, use_graph=False, t0=0.0, global_step=False):
        """One coarse step dt0 from time t0: subcycled (default) or, with
        global_step, one step dt0 of every level at once."""
        mk = ctypes.c_uint32(mask)
        flags = (STEP_GRAPH if use_graph else 0) | (STEP_GLOBAL if global_step else 0)
        check(_lib.load().af_amr_coarse_step(self.h, hier.h, self._pair(bufs), ctypes.byref(mk), float(t0),
                                             float(dt0), _ptr(flux_reg), int(flags), _stream()))
        return mk.value

    def amr_coarse_steps(self, hier, bufs, mask, dt0, nsteps, flux_reg, t0=0.0, global_step=False):
        """nsteps coarse steps dt0 from time t0 in one call (af_amr_coarse_steps):
        the result of nsteps amr_coarse_step calls, with one launch fewer per
        step on the batched path."""
        mk = ctypes.c_uint32(mask)
        flags = STEP_GLOBAL if global_step else 0
        check(_lib.load().af_amr_coarse_steps(self.h, hier.h, self._pair(bufs), ctypes.byref(mk), float(t0),
                                              float(dt0), int(nsteps), _ptr(flux_reg), int(flags), _stream()))
        return mk.value


    def amr_coarse_step_timed(self, hier, bufs, mask, dt0, flux_reg, events, t0=0.0):
        """af_amr_coarse_step_timed (a measurement helper): the subcycled
        coarse step with HIP event pairs recorded around its batched step
        launches.  events: raw hipEvent_t handles, two per launch.  Returns
        (mask, launches timed, cell-updates of each)."""
        n = len(events) // 2
        arr = (ctypes.c_void_p * max(1, 2 * n))(*events)
        cells = np.zeros(max(1, n))
        nl = ctypes.c_int32()
        mk = ctypes.c_uint32(mask)
        check(_lib.load().af_amr_coarse_step_timed(self.h, hier.h, self._pair(bufs), ctypes.byref(mk), float(t0),
                                                   float(dt0), _ptr(flux_reg), _stream(), arr, int(n),
                                                   ctypes.byref(nl), cells.ctypes.data_as(ctypes.c_void_p)))
        return mk.value, nl.value, cells[:nl.value].copy()


class Hierarchy:
    def __init__(self, ctx: Context, leaves=None, _handle=None):
        self.ctx = ctx
        L = _lib.load()
        if _handle is not None:
            self.h = _handle
        else:
            lv = np.ascontiguousarray([l[0] for l in leaves], dtype=np.int32)
            ix = np.ascontiguousarray([l[1] for l in leaves], dtype=np.int32)
            iy = np.ascontiguousarray([l[2] for l in leaves], dtype=np.int32)
            h = ctypes.c_void_p()
            check(L.af_hier_create(ctx.h, len(lv), lv.ctypes.data_as(ctypes.c_void_p),
                                   ix.ctypes.data_as(ctypes.c_void_p), iy.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.byref(h)))
            self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _lib.load().af_hier_destroy(self.h)
                self.h = None
        except Exception:  # interpreter shutdown
            pass

    def __len__(self):
        return _lib.load().af_hier_num_leaves(self.h)

    def leaves(self):
        n = len(self)
        lv, ix, iy = (np.zeros(n, np.int32) for _ in range(3))
        check(_lib.load().af_hier_get_leaves(self.h, lv.ctypes.data_as(ctypes.c_void_p),
                                             ix.ctypes.data_as(ctypes.c_void_p), iy.ctypes.data_as(ctypes.c_void_p)))
        return [(int(a), int(b), int(c)) for a, b, c in zip(lv, ix, iy)]

    def level_range(self, level):
        f, c = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().af_hier_level_range(self.h, int(level), ctypes.byref(f), ctypes.byref(c)))
        return f.value, c.value

    def finest(self):
        return _lib.load().af_hier_finest_level(self.h)

    def side_relations(self):
        rel = np.zeros((len(self), 4), np.int8)
        check(_lib.load().af_hier_side_relations(self.h, rel.ctypes.data_as(ctypes.c_void_p)))
        return rel

    def side_mask_ptr(self):
        return _lib.load().af_hier_side_mask(self.h)

    def leaf_xy_ptr(self):
        return _lib.load().af_hier_leaf_xy(self.h)

    def regrid(self, tags):
        t = np.ascontiguousarray(tags, dtype=np.int8)
        assert len(t) == len(self)
        h = ctypes.c_void_p()
        check(_lib.load().af_hier_regrid(self.ctx.h, self.h, t.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        return Hierarchy(self.ctx, _handle=h)


# ---------------------------------------------------------------------------
# host <-> state marshalling (layout conversion only)
# ---------------------------------------------------------------------------

def fma_probe(prec, nblocks=4096, iters=256):
    """Vector multiply-add rate of this device in TFLOP/s, measured with the
    library's probe kernel (af_fma_probe) timed by HIP events on torch's
    current stream."""
    torch = _torch()
    dt = torch.float32 if prec == FP32 else torch.float64
    out = torch.empty(nblocks * 256, dtype=dt, device="cuda")
    L = _lib.load()
    check(L.af_fma_probe(int(prec), _ptr(out), int(nblocks), int(iters), _stream()))  # warm-up
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    check(L.af_fma_probe(int(prec), _ptr(out), int(nblocks), int(iters), _stream()))
    e1.record()
    torch.cuda.synchronize()
    flops = 2.0 * 8 * 16 * iters * 256 * nblocks
    return flops / (e0.elapsed_time(e1) * 1e-3) / 1e12


def blocks_to_state(ctx: Context, blocks, npatch=None, pitch=None):
    """blocks: list over patches of dict kind -> [ncomp][m+5][m+5] arrays."""
    torch = _torch()
    npatch = npatch or len(blocks)
    t = ctx.new_state(npatch, pitch)
    S1 = ctx.prob.m + 5
    host = np.zeros((4, ctx.prob.ncomp, npatch, S1, t.shape[4]))
    for p, blk in enumerate(blocks):
        for k, kind in enumerate(KINDS):
            host[k, :, p, :, :S1] = blk[kind]
    t.copy_(torch.from_numpy(host).to(t.dtype))
    return t


def state_to_blocks(ctx: Context, t, npatch=None):
    S1 = ctx.prob.m + 5
    host = t.detach().double().cpu().numpy()
    n = npatch or t.shape[2]
    return [{kind: host[k, :, p, :, :S1].copy() for k, kind in enumerate(KINDS)} for p in range(n)]


class Tagger:
    """Learned regrid tagger (libaf.so af_cnn_*): BF16 matrix-core CNN with
    FP32 parameters and Adam."""

    NIN = 13

    def __init__(self, nin=NIN):
        L = _lib.load()
        h = ctypes.c_void_p()
        _lib.check_cnn(L.af_cnn_create(int(nin), ctypes.byref(h)))
        self.h = h
        self.nin = nin
        self.nparams = L.af_cnn_num_params(h)
        self.t = 0

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _lib.load().af_cnn_destroy(self.h)
                self.h = None
        except Exception:  # interpreter shutdown
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == self.nparams
        _lib.check_cnn(_lib.load().af_cnn_set_params(self.h, a.ctypes.data_as(ctypes.c_void_p)))
        self.t = 0

    def get_params(self):
        a = np.zeros(self.nparams, np.float32)
        _lib.check_cnn(_lib.load().af_cnn_get_params(self.h, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def set_normalization(self, mean, inv_std):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(inv_std, dtype=np.float32)
        _lib.check_cnn(_lib.load().af_cnn_set_normalization(self.h, m.ctypes.data_as(ctypes.c_void_p),
                                                             s.ctypes.data_as(ctypes.c_void_p)))

    def forward(self, x, acts=False):
        torch = _torch()
        B = x.shape[0]
        logits = torch.zeros((B, 3), dtype=torch.float32, device="cuda")
        a = torch.zeros((3, B * 256, 32), dtype=torch.float32, device="cuda") if acts else None
        _lib.check_cnn(_lib.load().af_cnn_forward(self.h, _ptr(x), int(B), _ptr(logits), _ptr(a), _stream()))
        return (logits, a) if acts else logits

    def loss_grad(self, x, labels, grad=None, dacts=False):
        """Loss (device [1]) and gradient (into grad, or the internal buffer);
        with dacts also each layer's upstream gradient [3][B*256][32]."""
        torch = _torch()
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        d = torch.zeros((3, x.shape[0] * 256, 32), dtype=torch.float32, device="cuda") if dacts else None
        _lib.check_cnn(_lib.load().af_cnn_loss_grad(self.h, _ptr(x), _ptr(labels), int(x.shape[0]), _ptr(loss),
                                                    _ptr(grad), _ptr(d), _stream()))
        return (loss, d) if dacts else loss

    def adam_step(self, lr, grad=None):
        self.t += 1
        _lib.check_cnn(_lib.load().af_cnn_adam_step(self.h, _ptr(grad), ctypes.c_float(lr), int(self.t), _stream()))

    def features(self, ctx, hier, bufs, mask):
        torch = _torch()
        x = torch.zeros((len(hier), self.nin, 16, 16), dtype=torch.float32, device="cuda")
        _lib.check_cnn(_lib.load().af_cnn_features(ctx.h, self.h, hier.h, ctx._pair(bufs), int(mask), _ptr(x),
                                                   _stream()))
        return x

    def tag(self, ctx, hier, bufs, mask, plain):
        torch = _torch()
        n = len(hier)
        tags = torch.zeros(n, dtype=torch.int8, device="cuda")
        learned = torch.zeros(n, dtype=torch.int8, device="cuda")
        _lib.check_cnn(_lib.load().af_cnn_tag(ctx.h, self.h, hier.h, ctx._pair(bufs), int(mask), _ptr(plain),
                                              _ptr(tags), _ptr(learned), _stream()))
        return tags, learned
