"""CPU oracle for the Active Flux patch step (TEST INFRASTRUCTURE ONLY).

A plain, single-threaded FP64 C++ implementation (af_oracle.cpp) of the
method of arXiv 2205.07572, loaded through ctypes.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
GPU library never does, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "af_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

D = ctypes.c_double
I = ctypes.c_int
P = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile the oracle: plain FP64, no contraction, no fast-math."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-shared",
                               "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.or_recon_eval.argtypes = [P, I, P, P, P]
        L.or_sector_mean.argtypes = [P, I, D, P]
        L.or_sector_mean.restype = D
        L.or_step_periodic.argtypes = [I, I, I, D, D, D, D, D, D, P, P, P, P]
        L.or_run_periodic.argtypes = [I, I, I, D, D, D, I, D, D, D, P, P, P, P]
        L.or_patch_step.argtypes = [I, I, I, D, D, D, D, D, D, I, P, P, P, P, P, P, P, P, P, I]
        L.or_run_periodic_rot.argtypes = [I, I, D, D, D, D, D, I, D, D, D, P, P, P, P]
        L.or_patch_step_rot.argtypes = [I, I, D, D, D, D, D, D, D, D, I, P, P, P, P, P, P, P, P, P, I]
        L.or_hier_set_rotation.argtypes = [P, D, D, D]
        L.or_run_periodic_swirl.argtypes = [I, I, D, D, D, D, D, I, D, P, P, P, P]
        L.or_patch_step_swirl.argtypes = [I, I, D, D, D, D, D, D, I, P, P, P, P, P, P, P, P, P, I]
        L.or_swirl_foot.argtypes = [D, D, D, D, D, D, P, P]
        L.or_patch_step_burgers.argtypes = [I, I, D, D, D, I, I, P, P, P, P, P, P, P, P, P, I]
        L.or_hier_set_swirl.argtypes = [P]
        L.or_hier_run_global.argtypes = [P, D, I]
        L.or_hier_set_time.argtypes = [P, D]
        L.or_hier_get_time.argtypes = [P]
        L.or_hier_get_time.restype = D
        L.or_hier_new.argtypes = [I, I, I, I, I, D, D, D, D, D, D, D]
        L.or_hier_new.restype = P
        L.or_hier_free.argtypes = [P]
        L.or_hier_set_leaves.argtypes = [P, I, P, P, P]
        L.or_hier_num_leaves.argtypes = [P]
        L.or_hier_num_leaves.restype = I
        L.or_hier_get_leaves.argtypes = [P, P, P, P]
        L.or_hier_set_block.argtypes = [P, I, I, P]
        L.or_hier_get_block.argtypes = [P, I, I, P]
        L.or_hier_get_reg.argtypes = [P, I, P]
        L.or_hier_set_reg.argtypes = [P, I, P]
        L.or_hier_side_relations.argtypes = [P, P]
        L.or_hier_fill.argtypes = [P, I, I]
        L.or_hier_step_level.argtypes = [P, I, D, I]
        L.or_hier_flux_correct.argtypes = [P, I]
        L.or_hier_coarse_step.argtypes = [P, D]
        L.or_hier_run.argtypes = [P, D, I]
        L.or_hier_tag.argtypes = [P, I, I, D, D, P, P]
        L.or_hier_regrid.argtypes = [P, P]
        L.or_hier_sum.argtypes = [P, P]
        L.or_hier_balanced.argtypes = [P]
        L.or_cnn_conv_backward.argtypes = [P, I, I, P, P, I, P, P, P]
        L.or_cnn_head.argtypes = [I, P, P, I, P, P, P, P, P]
        L.or_cnn_head.restype = D
        L.or_hier_balanced.restype = I
        L.or_refine_block.argtypes = [P, I, I, I, P, P, P, P]
        L.or_coarsen_block.argtypes = [P, P, P, P, P, P]
        L.or_cnn_num_params.argtypes = [I]
        L.or_cnn_num_params.restype = I
        L.or_cnn_forward.argtypes = [I, P, P, I, P, I, P]
        L.or_cnn_forward.restype = D
        L.or_cnn_grad.argtypes = [I, P, P, I, P, I, P, P]
        L.or_cnn_grad.restype = D
        L.or_round_bf16.argtypes = [D]
        L.or_round_bf16.restype = D
        L.or_cnn_conv.argtypes = [P, I, I, P, P, I, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


KINDS = ("avg", "corner", "xedge", "yedge")


def recon_eval(dofs9, xi, eta):
    """Evaluate one cell's reconstruction; dofs9 = [avg, c_ll, c_rl, c_lu,
    c_ru, e_l, e_r, e_b, e_t]."""
    d = np.ascontiguousarray(dofs9, dtype=np.float64)
    xi = np.ascontiguousarray(np.atleast_1d(xi), dtype=np.float64)
    eta = np.ascontiguousarray(np.atleast_1d(eta), dtype=np.float64)
    out = np.zeros_like(xi)
    lib().or_recon_eval(_p(d), len(xi), _p(xi), _p(eta), _p(out))
    return out


def sector_mean(coef4x4, quad, R):
    c = np.ascontiguousarray(coef4x4, dtype=np.float64).reshape(16)
    dm = np.zeros(1)
    m = lib().or_sector_mean(_p(c), int(quad), float(R), _p(dm))
    return m, dm[0]


def run_periodic(eq, dofs, dt, nsteps, a=0.0, b=0.0, c=1.0):
    """Advance a periodic grid (dict of [ncomp][ny][nx] arrays plus dx, dy)
    nsteps steps; returns a new dict."""
    out = {k: np.ascontiguousarray(dofs[k], dtype=np.float64).copy() for k in KINDS}
    ncomp, ny, nx = out["avg"].shape
    lib().or_run_periodic(int(eq), nx, ny, float(dofs["dx"]), float(dofs["dy"]), float(dt),
                          int(nsteps), float(a), float(b), float(c), _p(out["avg"]),
                          _p(out["corner"]), _p(out["xedge"]), _p(out["yedge"]))
    out["dx"], out["dy"] = dofs["dx"], dofs["dy"]
    return out


def run_periodic_rot(dofs, dt, nsteps, omega, xc=0.0, yc=0.0, x0=0.0, y0=0.0):
    """Solid-body rotation a = -omega (y - yc), b = omega (x - xc) (Sec. 4.2)
    on a periodic grid whose cell (0,0) has its lower-left corner at
    (x0, y0); returns a new dict."""
    out = {k: np.ascontiguousarray(dofs[k], dtype=np.float64).copy() for k in KINDS}
    _, ny, nx = out["avg"].shape
    lib().or_run_periodic_rot(nx, ny, float(x0), float(y0), float(dofs["dx"]), float(dofs["dy"]), float(dt),
                              int(nsteps), float(omega), float(xc), float(yc), _p(out["avg"]),
                              _p(out["corner"]), _p(out["xedge"]), _p(out["yedge"]))
    out["dx"], out["dy"] = dofs["dx"], dofs["dy"]
    return out


def patch_step_rot(m, block, x0p, y0p, dx, dy, dt, omega, xc=0.0, yc=0.0, region=0, flux4=None,
                   side_mask=0, g=2):
    """patch_step for solid-body rotation; (x0p, y0p) is the lower-left
    corner of the patch's cell (0,0)."""
    ins = {k: np.ascontiguousarray(block[k], dtype=np.float64) for k in KINDS}
    outs = {k: np.zeros_like(ins[k]) for k in KINDS}
    fp = _p(flux4) if flux4 is not None else None
    lib().or_patch_step_rot(int(m), int(g), float(x0p), float(y0p), float(dx), float(dy), float(dt),
                            float(omega), float(xc), float(yc), int(region), _p(ins["avg"]), _p(ins["corner"]),
                            _p(ins["xedge"]), _p(ins["yedge"]), _p(outs["avg"]), _p(outs["corner"]),
                            _p(outs["xedge"]), _p(outs["yedge"]), fp, int(side_mask))
    return outs


def run_periodic_swirl(dofs, dt, nsteps, t0=0.0, x0=0.0, y0=0.0):
    """Swirl flow of Sec. 4.3 on a periodic grid whose cell (0,0) has its
    lower-left corner at (x0, y0), from time t0; returns a new dict."""
    out = {k: np.ascontiguousarray(dofs[k], dtype=np.float64).copy() for k in KINDS}
    _, ny, nx = out["avg"].shape
    lib().or_run_periodic_swirl(nx, ny, float(x0), float(y0), float(dofs["dx"]), float(dofs["dy"]), float(dt),
                                int(nsteps), float(t0), _p(out["avg"]), _p(out["corner"]), _p(out["xedge"]),
                                _p(out["yedge"]))
    out["dx"], out["dy"] = dofs["dx"], dofs["dy"]
    return out


def patch_step_swirl(m, block, x0p, y0p, dx, dy, dt, t, region=0, flux4=None, side_mask=0, g=2):
    """patch_step for the swirl flow, the step starting at time t."""
    ins = {k: np.ascontiguousarray(block[k], dtype=np.float64) for k in KINDS}
    outs = {k: np.zeros_like(ins[k]) for k in KINDS}
    fp = _p(flux4) if flux4 is not None else None
    lib().or_patch_step_swirl(int(m), int(g), float(x0p), float(y0p), float(dx), float(dy), float(dt), float(t),
                              int(region), _p(ins["avg"]), _p(ins["corner"]), _p(ins["xedge"]), _p(ins["yedge"]),
                              _p(outs["avg"]), _p(outs["corner"]), _p(outs["xedge"]), _p(outs["yedge"]), fp,
                              int(side_mask))
    return outs


def patch_step_burgers(m, block, dx, dy, dt, iters=2, region=0, flux4=None, side_mask=0, g=2):
    """patch_step for Burgers' equation (Sec. 2.2) with `iters` fixed-point
    iterations per point value (the method uses two)."""
    ins = {k: np.ascontiguousarray(block[k], dtype=np.float64) for k in KINDS}
    outs = {k: np.zeros_like(ins[k]) for k in KINDS}
    fp = _p(flux4) if flux4 is not None else None
    lib().or_patch_step_burgers(int(m), int(g), float(dx), float(dy), float(dt), int(iters), int(region),
                                _p(ins["avg"]), _p(ins["corner"]), _p(ins["xedge"]), _p(ins["yedge"]),
                                _p(outs["avg"]), _p(outs["corner"]), _p(outs["xedge"]), _p(outs["yedge"]), fp,
                                int(side_mask))
    return outs


def swirl_foot(x, y, t, tau, dx, dy):
    """Foot of the swirl characteristic through (x, y) at t + tau, traced back
    to t by the oracle's Runge-Kutta step on a grid of spacing (dx, dy)."""
    fx, fy = ctypes.c_double(), ctypes.c_double()
    lib().or_swirl_foot(float(x), float(y), float(t), float(tau), float(dx), float(dy), ctypes.byref(fx),
                        ctypes.byref(fy))
    return fx.value, fy.value


def patch_step(eq, m, block, dx, dy, dt, region=0, a=0.0, b=0.0, c=1.0, flux4=None,
               side_mask=0, g=2):
    """One step on one patch block (dict kind -> [ncomp][S+1][S+1]).  Returns
    the output block; flux4 ([4][m][ncomp], float64) is accumulated if given."""
    ins = {k: np.ascontiguousarray(block[k], dtype=np.float64) for k in KINDS}
    outs = {k: np.zeros_like(ins[k]) for k in KINDS}
    fp = _p(flux4) if flux4 is not None else None
    lib().or_patch_step(int(eq), int(m), int(g), float(dx), float(dy), float(dt), float(a),
                        float(b), float(c), int(region), _p(ins["avg"]), _p(ins["corner"]),
                        _p(ins["xedge"]), _p(ins["yedge"]), _p(outs["avg"]),
                        _p(outs["corner"]), _p(outs["xedge"]), _p(outs["yedge"]), fp,
                        int(side_mask))
    return outs


class Hier:
    """Oracle AMR hierarchy: leaves (level, ix, iy) of m x m patches with two
    ghost layers on a periodic rectangle covered by n0x x n0y level-0
    patches."""

    def __init__(self, eq, m, n0x, n0y, lmax, x0=0.0, y0=0.0, lx=1.0, ly=1.0, a=0.0, b=0.0,
                 c=1.0, omega=0.0, xc=0.0, yc=0.0):
        """eq 0 advection (a, b), 1 acoustics (c), 2 solid-body rotation
        (omega about (xc, yc)), 3 the swirl flow of Sec. 4.3, 4 Burgers
        (Sec. 2.2)."""
        self.eq, self.m, self.n0x, self.n0y, self.lmax = eq, m, n0x, n0y, lmax
        self.x0, self.y0, self.lx, self.ly = x0, y0, lx, ly
        self.ncomp = 3 if eq == 1 else 1
        self.S1 = m + 5
        self.h = lib().or_hier_new(int(eq), int(m), int(n0x), int(n0y), int(lmax), float(x0),
                                   float(y0), float(lx), float(ly), float(a), float(b), float(c))
        if eq == 2:
            lib().or_hier_set_rotation(self.h, float(omega), float(xc), float(yc))
        elif eq == 3:
            lib().or_hier_set_swirl(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_hier_free(self.h)
            self.h = None

    def dx(self, level):
        return self.lx / (self.n0x * self.m) / 2 ** level

    def dy(self, level):
        return self.ly / (self.n0y * self.m) / 2 ** level

    def set_leaves(self, leaves):
        lv = np.array([l[0] for l in leaves], dtype=np.int32)
        ix = np.array([l[1] for l in leaves], dtype=np.int32)
        iy = np.array([l[2] for l in leaves], dtype=np.int32)
        lib().or_hier_set_leaves(self.h, len(leaves), lv.ctypes.data_as(P), ix.ctypes.data_as(P),
                                 iy.ctypes.data_as(P))

    def leaves(self):
        n = lib().or_hier_num_leaves(self.h)
        lv = np.zeros(n, np.int32); ix = np.zeros(n, np.int32); iy = np.zeros(n, np.int32)
        lib().or_hier_get_leaves(self.h, lv.ctypes.data_as(P), ix.ctypes.data_as(P),
                                 iy.ctypes.data_as(P))
        return [(int(a), int(b), int(c)) for a, b, c in zip(lv, ix, iy)]

    def set_block(self, leaf, block):
        for k, kind in enumerate(KINDS):
            arr = np.ascontiguousarray(block[kind], dtype=np.float64)
            assert arr.size == self.ncomp * self.S1 * self.S1
            lib().or_hier_set_block(self.h, int(leaf), k, _p(arr))

    def get_block(self, leaf):
        out = {}
        for k, kind in enumerate(KINDS):
            arr = np.zeros((self.ncomp, self.S1, self.S1))
            lib().or_hier_get_block(self.h, int(leaf), k, _p(arr))
            out[kind] = arr
        return out

    def get_reg(self, leaf):
        arr = np.zeros((4, self.m, self.ncomp))
        lib().or_hier_get_reg(self.h, int(leaf), _p(arr))
        return arr

    def set_reg(self, leaf, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        lib().or_hier_set_reg(self.h, int(leaf), _p(arr))

    def side_relations(self):
        n = lib().or_hier_num_leaves(self.h)
        rel = np.zeros((n, 4), np.int32)
        lib().or_hier_side_relations(self.h, rel.ctypes.data_as(P))
        return rel

    def init_from(self, data, nq=8):
        """Exact DOFs of `data` (afsynth.InitialData) on every leaf block."""
        import afsynth
        for k, (l, ix, iy) in enumerate(self.leaves()):
            dx, dy = self.dx(l), self.dy(l)
            blk = afsynth.dofs_block(data, self.m, 2, self.x0 + ix * self.m * dx,
                                     self.y0 + iy * self.m * dy, dx, dy, nq)
            self.set_block(k, blk)

    def fill(self, tmin=0, smin=0):
        lib().or_hier_fill(self.h, int(tmin), int(smin))

    def step_level(self, level, dt, region):
        lib().or_hier_step_level(self.h, int(level), float(dt), int(region))

    def flux_correct(self, level):
        lib().or_hier_flux_correct(self.h, int(level))

    def coarse_step(self, dt0):
        lib().or_hier_coarse_step(self.h, float(dt0))

    def run(self, dt0, nsteps):
        """nsteps subcycled coarse steps of dt0 (Sec. 3.2)."""
        lib().or_hier_run(self.h, float(dt0), int(nsteps))

    def run_global(self, dt, nsteps):
        """nsteps steps of dt on every level at once (no subcycling)."""
        lib().or_hier_run_global(self.h, float(dt), int(nsteps))

    @property
    def time(self):
        return lib().or_hier_get_time(self.h)

    @time.setter
    def time(self, t):
        lib().or_hier_set_time(self.h, float(t))

    def tag(self, mode, comp, theta_r, theta_c):
        n = lib().or_hier_num_leaves(self.h)
        tags = np.zeros(n, np.int8)
        vals = np.zeros(n)
        lib().or_hier_tag(self.h, int(mode), int(comp), float(theta_r), float(theta_c),
                          tags.ctypes.data_as(P), _p(vals))
        return tags, vals

    def regrid(self, tags):
        t = np.ascontiguousarray(tags, dtype=np.int8)
        assert len(t) == lib().or_hier_num_leaves(self.h)
        lib().or_hier_regrid(self.h, t.ctypes.data_as(P))

    def total(self):
        out = np.zeros(self.ncomp)
        lib().or_hier_sum(self.h, _p(out))
        return out

    def balanced(self):
        return bool(lib().or_hier_balanced(self.h))

    def refine_block(self, leaf, qx, qy):
        outs = {k: np.zeros((self.ncomp, self.S1, self.S1)) for k in KINDS}
        lib().or_refine_block(self.h, int(leaf), int(qx), int(qy), _p(outs["avg"]),
                              _p(outs["corner"]), _p(outs["xedge"]), _p(outs["yedge"]))
        return outs

    def coarsen_block(self, kids4):
        k4 = np.array(kids4, dtype=np.int32)
        outs = {k: np.zeros((self.ncomp, self.S1, self.S1)) for k in KINDS}
        lib().or_coarsen_block(self.h, k4.ctypes.data_as(P), _p(outs["avg"]),
                               _p(outs["corner"]), _p(outs["xedge"]), _p(outs["yedge"]))
        return outs


# ---------------------------------------------------------------------------
# learned tagger reference (not part of the paper's method)
# ---------------------------------------------------------------------------

def cnn_num_params(nin=13):
    return lib().or_cnn_num_params(int(nin))


def cnn_forward(params, x, labels=None, bf16=False):
    """x: [B][nin][16][16]; returns (logits [B][3], mean cross-entropy)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    B, nin = xx.shape[0], xx.shape[1]
    logits = np.zeros((B, 3))
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
    loss = lib().or_cnn_forward(nin, _p(p), _p(xx), B, lab.ctypes.data_as(P) if lab is not None else None,
                                int(bf16), _p(logits))
    return logits, loss


def cnn_grad(params, x, labels, bf16=False, want_acts=False):
    """Gradient of the mean cross-entropy; optionally the activations of
    sample 0 ([z1, a1, z2, a2, z3, a3], each [32][16][16])."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    B, nin = xx.shape[0], xx.shape[1]
    g = np.zeros_like(p)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    acts = np.zeros((6, 32, 16, 16)) if want_acts else None
    loss = lib().or_cnn_grad(nin, _p(p), _p(xx), B, lab.ctypes.data_as(P), int(bf16), _p(g),
                             _p(acts) if acts is not None else None)
    return (loss, g, acts) if want_acts else (loss, g)


def round_bf16(v):
    return lib().or_round_bf16(float(v))


def cnn_conv_backward(x, w, dz, bf16=False):
    """Adjoint of one 3x3 convolution layer: x [B][cin][16][16] its input, dz
    [B][32][16][16] the gradient with respect to its pre-activation.
    Returns (gW [32][cin][3][3], gb [32], dx [B][cin][16][16])."""
    xx = np.ascontiguousarray(x, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    dd = np.ascontiguousarray(dz, dtype=np.float64)
    B, cin = xx.shape[0], xx.shape[1]
    gW = np.zeros((32, cin, 3, 3))
    gb = np.zeros(32)
    dx = np.zeros_like(xx)
    lib().or_cnn_conv_backward(_p(xx), B, cin, _p(ww), _p(dd), int(bf16), _p(gW), _p(gb), _p(dx))
    return gW, gb, dx


def cnn_head(params, a3, labels):
    """Pooling, head and softmax cross-entropy from the last layer's
    post-activation a3 [B][32][16][16]: (loss, logits [B][3], gWh [3][32],
    gbh [3], da3 [B][32][16][16])."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    aa = np.ascontiguousarray(a3, dtype=np.float64)
    B = aa.shape[0]
    nin = _nin_of(p.size)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    logits = np.zeros((B, 3))
    gWh = np.zeros((3, 32))
    gbh = np.zeros(3)
    da3 = np.zeros_like(aa)
    loss = lib().or_cnn_head(nin, _p(p), _p(aa), B, lab.ctypes.data_as(P), _p(logits), _p(gWh), _p(gbh), _p(da3))
    return loss, logits, gWh, gbh, da3


def _nin_of(nparams):
    for nin in range(1, 33):
        if cnn_num_params(nin) == nparams:
            return nin
    raise ValueError("parameter count matches no input width")


def cnn_conv(x, w, b, bf16=False):
    """One 3x3 convolution plus bias: x [B][cin][16][16] -> [B][32][16][16]."""
    xx = np.ascontiguousarray(x, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros((xx.shape[0], 32, 16, 16))
    lib().or_cnn_conv(_p(xx), xx.shape[0], xx.shape[1], _p(ww), _p(bb), int(bf16), _p(out))
    return out
