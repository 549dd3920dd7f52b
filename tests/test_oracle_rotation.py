"""Oracle pins for solid-body rotation (Sec. 4.2): a = -pi y, b = pi x on
[-1, 1]^2, point values by tracing the characteristic circles back exactly,
Simpson fluxes with the velocity at each node."""
import numpy as np
import pytest

import afsynth
import oracle

OMEGA = np.pi
KINDS = ("avg", "corner", "xedge", "yedge")


def _grid(data, N, nq=4):
    """Exact DOFs on the N x N grid of [-1, 1]^2 (cell (0,0) at (-1, -1))."""
    return afsynth.dofs_periodic(data, N, N, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, nq=nq)


def _dt(N, cfl):
    # largest speed in either direction is omega * 1 on [-1, 1]^2
    return cfl * (2.0 / N) / OMEGA


def test_point_values_are_the_back_rotated_data_for_biquadratics():
    """One step of a patch block holding exact DOFs of a biquadratic: every new
    point value equals q0 at the node turned back by -omega tau (the
    reconstruction is exact for biquadratics), for both time levels used in
    the flux (checked through dt/2 and dt runs)."""
    m, g = 8, 2
    x0p, y0p = -0.3, 0.1
    dx = dy = 0.05
    coeffs = {(0, 0): 0.3, (1, 0): 0.7, (0, 1): -0.4, (2, 0): 0.25, (1, 1): -0.6, (0, 2): 0.35,
              (2, 1): 0.2, (1, 2): -0.15, (2, 2): 0.1}
    data = afsynth.polynomial([coeffs])
    blk = afsynth.dofs_block(data, m, g, x0p, y0p, dx, dy, 6)
    rot = afsynth.solid_body(lambda x, y: data.f(x, y)[0], OMEGA)
    for tau in (0.004, 0.011):
        out = oracle.patch_step_rot(m, blk, x0p, y0p, dx, dy, tau, OMEGA)
        loc = np.arange(m + 1)
        xn, yn = x0p + loc * dx, y0p + loc * dy
        X, Y = np.meshgrid(xn, yn)
        want = rot.exact(X, Y, tau)[0]
        got = out["corner"][0, g:g + m + 1, g:g + m + 1]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
        Xe, Ye = np.meshgrid(xn, yn[:-1] + 0.5 * dy)
        np.testing.assert_allclose(out["xedge"][0, g:g + m, g:g + m + 1], rot.exact(Xe, Ye, tau)[0], rtol=0,
                                   atol=1e-13)
        Xy, Yy = np.meshgrid(xn[:-1] + 0.5 * dx, yn)
        np.testing.assert_allclose(out["yedge"][0, g:g + m + 1, g:g + m], rot.exact(Xy, Yy, tau)[0], rtol=0,
                                   atol=1e-13)


def test_rotation_direction_and_period():
    """A narrow bump at (0.5, 0) moves counter-clockwise: after a quarter turn
    (t = 1/2) it sits at (0, 0.5)."""
    N = 64
    data = afsynth.solid_body(afsynth.gauss_q0(0.5, 0.0, 200.0), OMEGA)
    d0 = _grid(data, N)
    n = int(round(0.5 / _dt(N, 0.6)))
    out = oracle.run_periodic_rot(d0, 0.5 / n, n, OMEGA, x0=-1.0, y0=-1.0)
    j, i = np.unravel_index(np.argmax(out["avg"][0]), (N, N))
    xc, yc = -1.0 + (i + 0.5) * 2.0 / N, -1.0 + (j + 0.5) * 2.0 / N
    assert abs(xc) < 2.0 / N and abs(yc - 0.5) < 2.0 / N


def test_constant_state_preserved_uniform():
    """Remark of Sec. 4.2: fluxes in x depend on y only and in y on x only, so
    the flux differences cancel and a constant state is kept."""
    N = 32
    d0 = {k: np.full((1, N, N), 0.7) for k in KINDS}
    d0["dx"] = d0["dy"] = 2.0 / N
    out = oracle.run_periodic_rot(d0, _dt(N, 0.9), 40, OMEGA, x0=-1.0, y0=-1.0)
    for k in KINDS:
        assert np.abs(out[k] - 0.7).max() <= 1e-14, k


def test_constant_state_preserved_with_subcycling():
    """The same on a diagonally refined hierarchy with subcycling and the
    conservative fix: the fill reproduces constants and the fine fluxes of a
    constant state sum to the coarse one (Simpson is exact for the linear
    velocity)."""
    m, n0, lc = 8, 2, 1
    h = oracle.Hier(2, m, n0, n0, lc + 1, x0=-1.0, y0=-1.0, lx=2.0, ly=2.0, omega=OMEGA)
    h.set_leaves(afsynth.diagonal_leaves(n0, lc))
    h.init_from(afsynth.polynomial([{(0, 0): 0.7}]), nq=2)
    dt0 = 0.9 * h.dx(0) / OMEGA
    h.run(dt0, 6)
    for k in range(len(h.leaves())):
        b = h.get_block(k)
        assert np.abs(b["avg"][0, 2:2 + m, 2:2 + m] - 0.7).max() <= 1e-13


def test_conservation():
    """Periodic sum of the averages is kept to round-off (data vanish near
    the boundary, where the rotation field is not periodic)."""
    N = 48
    data = afsynth.solid_body(afsynth.gauss_q0(0.2, 0.1, 100.0), OMEGA)  # below 1e-27 on the boundary
    d0 = _grid(data, N)
    out = oracle.run_periodic_rot(d0, _dt(N, 0.8), 30, OMEGA, x0=-1.0, y0=-1.0)
    s0, s1 = d0["avg"].sum(), out["avg"].sum()
    assert abs(s1 - s0) <= 1e-13 * np.abs(d0["avg"]).sum()


def test_third_order_convergence():
    """L1 error of the averages after a quarter turn of a smooth Gaussian
    against the exactly rotated data: EOC 64 -> 128 near 3."""
    data = afsynth.solid_body(afsynth.gauss_q0(0.25, 0.0, 50.0), OMEGA)  # below 1e-12 on the boundary
    T = 0.5
    errs = []
    for N in (32, 64, 128):
        d0 = _grid(data, N)
        n = int(np.ceil(T / _dt(N, 0.6)))
        out = oracle.run_periodic_rot(d0, T / n, n, OMEGA, x0=-1.0, y0=-1.0)
        ex = afsynth.InitialData(1, lambda x, y: data.exact(x, y, T))
        ref = _grid(ex, N)
        errs.append(np.abs(out["avg"] - ref["avg"]).sum() * (2.0 / N) ** 2)
    eoc = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("rotation L1", errs, "EOC", eoc)
    assert 2.7 <= eoc[1] <= 3.3, eoc
