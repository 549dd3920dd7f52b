"""Seeded synthetic inputs for the Active Flux workloads.

This module produces initial degrees of freedom (exact point values and cell
averages of analytic initial data), exact reference solutions, refinement
layouts and random numbers.  It holds none of the Active Flux method's own
arithmetic (no reconstruction, evolution, flux or update), so that both the
CPU oracle and the GPU library can be fed from it without sharing method code.

DOF conventions (Sec. 2 of the paper, cell ownership): cell (i,j) owns its
average, the corner (x_{i-1/2}, y_{j-1/2}), the left-edge midpoint
(x_{i-1/2}, y_j) and the bottom-edge midpoint (x_i, y_{j-1/2}).

Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), uniform doubles
(x >> 11) * 2^-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (published algorithm), uniform doubles in [0,1)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (2.0 ** -53))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1))


# ---------------------------------------------------------------------------
# Quadrature for cell averages of analytic data
# ---------------------------------------------------------------------------

def gauss_legendre(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def cell_averages(f, xc, yc, dx, dy, ncomp, nq=8):
    """Cell averages of f over cells centred at (xc, yc) (arrays of equal
    shape) by nq x nq Gauss-Legendre quadrature; f(x, y) returns an array of
    shape (ncomp,) + x.shape."""
    gx, gw = gauss_legendre(nq)
    out = np.zeros((ncomp,) + np.shape(xc))
    for a in range(nq):
        for b in range(nq):
            x = xc + 0.5 * dx * gx[a]
            y = yc + 0.5 * dy * gx[b]
            out += 0.25 * gw[a] * gw[b] * np.asarray(f(x, y)).reshape((ncomp,) + np.shape(xc))
    return out


# ---------------------------------------------------------------------------
# Initial data
# ---------------------------------------------------------------------------

@dataclass
class InitialData:
    """An analytic field f(x, y) -> (ncomp, ...) array."""
    ncomp: int
    f: object
    exact: object = None  # exact(x, y, t) -> (ncomp, ...) or None

    def __call__(self, x, y):
        return self.f(x, y)


def _periodic_gauss(x, y, x0, y0, alpha, lx=1.0, ly=1.0):
    """exp(-alpha |x - x0|^2) summed over the 3x3 periodic images."""
    s = 0.0
    for ox in (-lx, 0.0, lx):
        for oy in (-ly, 0.0, ly):
            s = s + np.exp(-alpha * ((x - x0 - ox) ** 2 + (y - y0 - oy) ** 2))
    return s


def sinsin_bump(a=1.0, b=0.5):
    """q0 = sin(2 pi x) sin(2 pi y) + exp(-100 |x - (0.5,0.5)|^2), periodic on
    the unit square (bump periodised over its images); advected with (a,b)."""

    def q0(x, y):
        return (np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) +
                _periodic_gauss(x, y, 0.5, 0.5, 100.0))[None]

    def exact(x, y, t):
        return q0(np.mod(x - a * t, 1.0), np.mod(y - b * t, 1.0))

    return InitialData(1, q0, exact)


def fourier_modes(seed: int, nmodes: int = 8, kmax: int = 8, a=1.0, b=0.5):
    """Seeded sum of nmodes plane waves A sin(2 pi (k x + l y) + phi) with
    A ~ U(-1,1), (k,l) ~ U{-kmax..kmax}^2 minus (0,0), phi ~ U[0, 2 pi)."""
    rng = SplitMix64(0xA5F0 + seed)
    modes = []
    while len(modes) < nmodes:
        A = rng.uniform(-1.0, 1.0)
        k = rng.randint(-kmax, kmax)
        l = rng.randint(-kmax, kmax)
        phi = rng.uniform(0.0, 2 * np.pi)
        if k == 0 and l == 0:
            continue
        modes.append((A, k, l, phi))

    def q0(x, y):
        s = 0.0
        for A, k, l, phi in modes:
            s = s + A * np.sin(2 * np.pi * (k * x + l * y) + phi)
        return np.asarray(s)[None] * np.ones_like(x)[None]

    def exact(x, y, t):
        return q0(x - a * t, y - b * t)

    return InitialData(1, q0, exact)


def tanh_disc(r0=0.15, width=0.02, xc=0.5, yc=0.5, a=1.0, b=0.5):
    """Smoothed disc of Sec. 4.1: H(r + r0) - H(r - r0), H(r) = (tanh(r/w)+1)/2."""

    def H(r):
        return 0.5 * (np.tanh(r / width) + 1.0)

    def q0(x, y):
        r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
        return (H(r + r0) - H(r - r0))[None]

    def exact(x, y, t):
        return q0(np.mod(x - a * t, 1.0), np.mod(y - b * t, 1.0))

    return InitialData(1, q0, exact)


def lukacova(c=1.0):
    """Acoustic test of Sec. 4.5.1 on [-1,1]^2 with its exact solution."""

    def exact(x, y, t):
        x = np.asarray(x, dtype=float)
        p = -np.cos(2 * np.pi * c * t) * (np.sin(2 * np.pi * x) + np.sin(2 * np.pi * y)) / c
        u = np.sin(2 * np.pi * c * t) * np.cos(2 * np.pi * x) / c + 0 * y
        v = np.sin(2 * np.pi * c * t) * np.cos(2 * np.pi * y) / c + 0 * x
        return np.stack([p, u, v])

    return InitialData(3, lambda x, y: exact(x, y, 0.0), exact)


def gaussian_pulse(seed: int, alpha=200.0):
    """p0 = exp(-alpha |x - x0|^2) (periodised), u = v = 0, x0 ~ U[0,1)^2."""
    rng = SplitMix64(0xC0FFEE + seed)
    x0, y0 = rng.uniform(), rng.uniform()

    def f(x, y):
        p = _periodic_gauss(x, y, x0, y0, alpha)
        z = np.zeros_like(p)
        return np.stack([p, z, z])

    d = InitialData(3, f)
    d.center = (x0, y0)
    return d


WAVE_VECTORS = [(40, 0), (-40, 0), (0, 40), (0, -40), (24, 32), (-24, 32), (24, -32),
                (-24, -32), (32, 24), (-32, 24), (32, -24), (-32, -24)]


def wave_packet(seed: int, alpha=50.0, kdiv=1):
    """p0 = exp(-alpha |x - x0|^2) cos(k . x), |k| = 80 pi / kdiv with k in
    2 pi Z^2 (so the data is periodic; kdiv in {1, 2, 4, 8} keeps the lattice
    vectors integral), direction and x0 from the seed; u = v = 0."""
    assert kdiv in (1, 2, 4, 8)
    rng = SplitMix64(0xBEEF + seed)
    x0, y0 = rng.uniform(), rng.uniform()
    kx, ky = WAVE_VECTORS[rng.randint(0, len(WAVE_VECTORS) - 1)]
    kx, ky = 2 * np.pi * (kx // kdiv), 2 * np.pi * (ky // kdiv)

    def f(x, y):
        p = _periodic_gauss(x, y, x0, y0, alpha) * np.cos(kx * x + ky * y)
        z = np.zeros_like(p)
        return np.stack([p, z, z])

    d = InitialData(3, f)
    d.center = (x0, y0)
    d.k = (kx, ky)
    return d


def solid_body(q0, omega=np.pi, xc=0.0, yc=0.0):
    """Data q0(x, y) (scalar function) under solid-body rotation
    a = -omega (y - yc), b = omega (x - xc) (Sec. 4.2): the exact solution at
    time t is q0 at the point turned back by -omega t about (xc, yc)."""

    def f(x, y):
        return np.asarray(q0(np.asarray(x, float), np.asarray(y, float)))[None]

    def exact(x, y, t):
        c, s = np.cos(omega * t), np.sin(omega * t)
        rx, ry = np.asarray(x, float) - xc, np.asarray(y, float) - yc
        return f(xc + rx * c + ry * s, yc - rx * s + ry * c)

    return InitialData(1, f, exact)


def disc_q0(r0=0.15, width=0.02, xc=0.5, yc=0.5):
    """The smoothed disc H(r + r0) - H(r - r0), H(r) = (tanh(r/w)+1)/2, of
    eq. AdvH as a plain function of (x, y) (not periodised)."""

    def q0(x, y):
        r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
        return 0.5 * (np.tanh((r + r0) / width) - np.tanh((r - r0) / width))

    return q0


def swirl_gaussians():
    """Initial data eq. id_swirl of the swirl test (Sec. 4.3): two Gaussians
    exp(-100 |x - (0.5, 0.25)|^2) + exp(-100 |x - (0.5, 0.75)|^2) on the
    periodic unit square, periodised over the 3x3 images.  The swirl field
    reverses at t = 1/2, so at t = 1 the exact solution is the initial data."""

    def q0(x, y):
        return (_periodic_gauss(x, y, 0.5, 0.25, 100.0) + _periodic_gauss(x, y, 0.5, 0.75, 100.0))[None]

    def exact(x, y, t):
        if abs(t - round(t)) > 1e-12:
            raise ValueError("the swirl solution is known in closed form at integer times only")
        return q0(x, y)

    return InitialData(1, q0, exact)


def burgers_sinsin(amp=1.0, shift=0.1):
    """Initial data eq. sinsin01 of the Burgers test (Sec. 4.4):
    q0 = amp sin(2 pi x) sin(2 pi y) + shift on the periodic unit square.

    The exact solution of q_t + (q^2/2)_x + (q^2/2)_y = 0 for smooth times
    is the implicit q = q0(x - q t, y - q t) (characteristics along (1, 1)
    carrying q).  Along s = x + y the data's slope is at most 2 pi amp, so
    characteristics first cross at t* = 1 / (2 pi amp) (0.159 for amp = 1);
    `exact` solves the relation by Newton's method for t < t*."""

    def q0(x, y):
        return (amp * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) + shift)[None]

    def exact(x, y, t):
        if t * 2 * np.pi * amp >= 1.0:
            raise ValueError("the Burgers solution is smooth only before t* = 1 / (2 pi amp)")
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        q = q0(x, y)[0]
        for _ in range(60):
            u, v = x - q * t, y - q * t
            su, cu = np.sin(2 * np.pi * u), np.cos(2 * np.pi * u)
            sv, cv = np.sin(2 * np.pi * v), np.cos(2 * np.pi * v)
            F = q - (amp * su * sv + shift)
            dF = 1.0 + t * 2 * np.pi * amp * (cu * sv + su * cv)
            dq = F / dF
            q = q - dq
            if np.abs(dq).max() < 1e-15:
                break
        return q[None]

    return InitialData(1, q0, exact)


def gauss_q0(x0, y0, alpha):
    """exp(-alpha |x - x0|^2) as a plain function of (x, y)."""
    return lambda x, y: np.exp(-alpha * ((x - x0) ** 2 + (y - y0) ** 2))


def polynomial(coeffs, ncomp=1):
    """Polynomial data sum c[m][n] x^m y^n per component (coeffs: list of
    dicts {(m,n): c}); used for exactness checks."""

    def f(x, y):
        x = np.asarray(x, dtype=float)
        out = []
        for cc in coeffs:
            s = np.zeros_like(x, dtype=float) + 0.0 * np.asarray(y, dtype=float)
            for (m, n), c in cc.items():
                s = s + c * x ** m * np.asarray(y, dtype=float) ** n
            out.append(s)
        return np.stack(out)

    return InitialData(ncomp, f)


# ---------------------------------------------------------------------------
# DOF arrays
# ---------------------------------------------------------------------------

def dofs_periodic(data: InitialData, nx, ny, x0=0.0, y0=0.0, lx=1.0, ly=1.0, nq=8):
    """Exact DOFs on a periodic nx x ny grid; arrays [ncomp][ny][nx] for
    avg, corner, xedge, yedge."""
    dx, dy = lx / nx, ly / ny
    i = np.arange(nx)
    j = np.arange(ny)
    I, J = np.meshgrid(i, j)  # [ny][nx]
    xc = x0 + (I + 0.5) * dx
    yc = y0 + (J + 0.5) * dy
    avg = cell_averages(data.f, xc, yc, dx, dy, data.ncomp, nq)
    corner = np.asarray(data.f(xc - 0.5 * dx, yc - 0.5 * dy)).reshape(avg.shape)
    xedge = np.asarray(data.f(xc - 0.5 * dx, yc)).reshape(avg.shape)
    yedge = np.asarray(data.f(xc, yc - 0.5 * dy)).reshape(avg.shape)
    return {"avg": avg, "corner": corner, "xedge": xedge, "yedge": yedge,
            "dx": dx, "dy": dy}


def block_positions(m, g, x0p, y0p, dx, dy):
    """Physical positions of every entry of the (m+2g+1)^2 block planes, for
    a patch whose interior starts at (x0p, y0p).  Returns dict kind ->
    (x, y, valid-mask)."""
    S1 = m + 2 * g + 1
    loc = np.arange(S1) - g  # local index of row/col
    I, J = np.meshgrid(loc, loc)  # [row j][col i]
    out = {}
    out["avg"] = (x0p + (I + 0.5) * dx, y0p + (J + 0.5) * dy, (I < m + g) & (J < m + g))
    out["corner"] = (x0p + I * dx, y0p + J * dy, np.ones_like(I, dtype=bool))
    out["xedge"] = (x0p + I * dx, y0p + (J + 0.5) * dy, J < m + g)
    out["yedge"] = (x0p + (I + 0.5) * dx, y0p + J * dy, I < m + g)
    return out


def dofs_block(data: InitialData, m, g, x0p, y0p, dx, dy, nq=8):
    """Exact DOFs on one patch block (interior and ghost layers), arrays
    [ncomp][S+1][S+1] for avg, corner, xedge, yedge (unused entries 0)."""
    pos = block_positions(m, g, x0p, y0p, dx, dy)
    res = {}
    for kind, (x, y, valid) in pos.items():
        if kind == "avg":
            v = cell_averages(data.f, x, y, dx, dy, data.ncomp, nq)
        else:
            v = np.asarray(data.f(x, y)).reshape((data.ncomp,) + x.shape)
        res[kind] = np.where(valid[None], v, 0.0)
    return res


def periodic_to_blocks(dofs, m, g=2):
    """Cut a periodic grid's DOFs ([ncomp][ny][nx]) into patch blocks of m x m
    cells with g ghost layers filled by periodic wrap.  Returns dict kind ->
    [npy*npx][ncomp][S+1][S+1] (patch order: row-major, iy then ix)."""
    ncomp, ny, nx = dofs["avg"].shape
    npx, npy = nx // m, ny // m
    S1 = m + 2 * g + 1
    loc = np.arange(S1) - g
    out = {k: np.zeros((npx * npy, ncomp, S1, S1)) for k in ("avg", "corner", "xedge", "yedge")}
    for py in range(npy):
        for px in range(npx):
            gi = (px * m + loc) % nx
            gj = (py * m + loc) % ny
            for k in out:
                out[k][py * npx + px] = dofs[k][:, gj[:, None], gi[None, :]]
            out["avg"][py * npx + px][:, m + g:, :] = 0.0
            out["avg"][py * npx + px][:, :, m + g:] = 0.0
            out["xedge"][py * npx + px][:, m + g:, :] = 0.0
            out["yedge"][py * npx + px][:, :, m + g:] = 0.0
    return out


def blocks_interior(blocks, m, g=2):
    """Inverse of periodic_to_blocks for the owned DOFs: returns periodic
    arrays [ncomp][ny][nx]."""
    P = blocks["avg"].shape[0]
    ncomp = blocks["avg"].shape[1]
    npx = int(round(math.sqrt(P)))
    npy = P // npx
    out = {}
    for k in ("avg", "corner", "xedge", "yedge"):
        arr = np.zeros((ncomp, npy * m, npx * m))
        for py in range(npy):
            for px in range(npx):
                arr[:, py * m:(py + 1) * m, px * m:(px + 1) * m] = blocks[k][py * npx + px][:, g:g + m, g:g + m]
        out[k] = arr
    return out


# ---------------------------------------------------------------------------
# Refinement layouts (lists of leaves (level, ix, iy))
# ---------------------------------------------------------------------------

def uniform_leaves(n0x, n0y, level):
    return [(level, ix, iy) for iy in range(n0y << level) for ix in range(n0x << level)]


def diagonal_leaves(n0, lcoarse):
    """Level lcoarse everywhere, with the patches that meet the diagonal
    y = x refined once (static diagonal refinement as in Sec. 4.1 and 4.5.1);
    the result is 2:1 corner balanced by construction (one level step)."""
    n = n0 << lcoarse
    leaves = []
    for iy in range(n):
        for ix in range(n):
            if ix == iy:
                for q in range(4):
                    leaves.append((lcoarse + 1, 2 * ix + (q & 1), 2 * iy + (q >> 1)))
            else:
                leaves.append((lcoarse, ix, iy))
    return sorted(leaves, key=lambda t: (t[0], t[2], t[1]))


def antidiagonal_leaves(n0, lcoarse):
    """Level lcoarse everywhere, with the patches on the diagonal from the
    upper-left to the lower-right patch refined once (the static layout of
    the Burgers test, Sec. 4.4)."""
    n = n0 << lcoarse
    leaves = []
    for iy in range(n):
        for ix in range(n):
            if ix + iy == n - 1:
                for q in range(4):
                    leaves.append((lcoarse + 1, 2 * ix + (q & 1), 2 * iy + (q >> 1)))
            else:
                leaves.append((lcoarse, ix, iy))
    return sorted(leaves, key=lambda t: (t[0], t[2], t[1]))


def sort_leaves(leaves):
    return sorted(leaves, key=lambda t: (t[0], t[2], t[1]))


# ---------------------------------------------------------------------------
# Exact acoustic solutions on the periodic unit square by Fourier series
# ---------------------------------------------------------------------------

class FourierAcoustics:
    """Exact solution of p_t + c div u = 0, u_t + c grad p = 0 on the periodic
    unit square for u(0) = 0 and p(0) = sum_k phat_k e^{i k.x}:
      p = sum phat_k cos(c|k|t) e^{ik.x},
      u = -sum i (k/|k|) phat_k sin(c|k|t) e^{ik.x}.
    Modes are given on a tensor grid k = 2 pi (a, b), |a|,|b| <= nmax.  Values
    on tensor products of coordinates are evaluated as small matrix products;
    cell averages multiply each mode by sinc(k dx/2) sinc(k dy/2)."""

    def __init__(self, phat, nmax, c=1.0):
        self.phat = phat  # complex [2nmax+1][2nmax+1], index [a][b] for kx = 2 pi a, ky = 2 pi b
        self.nmax = nmax
        self.c = c
        n = np.arange(-nmax, nmax + 1)
        self.kx = 2 * np.pi * n

    def _coeffs(self, t):
        KX, KY = np.meshgrid(self.kx, self.kx, indexing="ij")
        K = np.sqrt(KX ** 2 + KY ** 2)
        Ksafe = np.where(K == 0, 1.0, K)
        cp = self.phat * np.cos(self.c * K * t)
        s = self.phat * np.sin(self.c * K * t)
        cu = -1j * (KX / Ksafe) * s
        cv = -1j * (KY / Ksafe) * s
        return cp, cu, cv

    def grid_values(self, xs, ys, t, dx=None, dy=None):
        """(3, len(ys), len(xs)) values at the tensor grid (xs, ys); with dx, dy
        given, averages over cells of that size centred there."""
        fx = np.exp(1j * np.outer(xs, self.kx))  # [nx][K]
        fy = np.exp(1j * np.outer(ys, self.kx))
        if dx is not None:
            fx = fx * np.sinc(self.kx * dx / 2 / np.pi)[None]
            fy = fy * np.sinc(self.kx * dy / 2 / np.pi)[None]
        out = []
        for C in self._coeffs(t):
            out.append(np.real(fy @ C.T @ fx.T))  # [ny][nx]
        return np.stack(out)

    def block(self, m, g, x0p, y0p, dx, dy, t):
        """DOFs of one patch block at time t, as afsynth.dofs_block lays them out."""
        S1 = m + 2 * g + 1
        loc = np.arange(S1) - g
        xn, yn = x0p + loc * dx, y0p + loc * dy
        xc, yc = xn + 0.5 * dx, yn + 0.5 * dy
        res = {"avg": self.grid_values(xc, yc, t, dx, dy), "corner": self.grid_values(xn, yn, t),
               "xedge": self.grid_values(xn, yc, t), "yedge": self.grid_values(xc, yn, t)}
        last = m + 2 * g  # the outer node line has no cell
        res["avg"][:, last:, :] = 0.0
        res["avg"][:, :, last:] = 0.0
        res["xedge"][:, last:, :] = 0.0
        res["yedge"][:, :, last:] = 0.0
        return res


def gaussian_pulse_exact(d: InitialData, alpha=200.0, c=1.0, nmax=28):
    """Fourier-series exact solution of gaussian_pulse (phat_k = (pi/alpha)
    e^{-|k|^2/(4 alpha)} e^{-i k.x0})."""
    x0, y0 = d.center
    n = np.arange(-nmax, nmax + 1)
    KX, KY = np.meshgrid(2 * np.pi * n, 2 * np.pi * n, indexing="ij")
    phat = (np.pi / alpha) * np.exp(-(KX ** 2 + KY ** 2) / (4 * alpha)) * np.exp(-1j * (KX * x0 + KY * y0))
    return FourierAcoustics(phat, nmax, c)


def wave_packet_exact(d: InitialData, alpha=50.0, c=1.0, half_width=14):
    """Fourier-series exact solution of wave_packet: phat_k = (G(k-k0) +
    G(k+k0))/2 with G the transform of the periodised Gaussian centred at x0,
    modes within half_width of +-k0 (in units of 2 pi)."""
    x0, y0 = d.center
    k0x, k0y = d.k
    a0, b0 = int(round(k0x / (2 * np.pi))), int(round(k0y / (2 * np.pi)))
    nmax = max(abs(a0), abs(b0)) + half_width
    n = np.arange(-nmax, nmax + 1)
    KX, KY = np.meshgrid(2 * np.pi * n, 2 * np.pi * n, indexing="ij")

    def g(qx, qy):
        return (np.pi / alpha) * np.exp(-(qx ** 2 + qy ** 2) / (4 * alpha))

    ph0 = np.exp(1j * (k0x * x0 + k0y * y0))  # transform of g e^{ik0.x} is ghat(k-k0) e^{-i(k-k0).x0}
    phat = 0.5 * (g(KX - k0x, KY - k0y) * ph0 + g(KX + k0x, KY + k0y) / ph0) * np.exp(-1j * (KX * x0 + KY * y0))
    return FourierAcoustics(phat, nmax, c)
