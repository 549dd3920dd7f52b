"""Oracle pins for the swirl flow (Sec. 4.3): stream function
Psi = sin^2(pi x) sin^2(pi y) cos(pi t) / pi, velocities by centred
differences of Psi over one cell (eq. swirlODE), feet by one classical
Runge-Kutta step backwards in time, fluxes with the face-midpoint velocity at
each Simpson time (eq. swirlF, swirlG)."""
import numpy as np

import afsynth
import oracle

KINDS = ("avg", "corner", "xedge", "yedge")


def _vel(x, y, t, dx, dy):
    # eq. swirlODE, written out independently of the oracle
    psi = lambda x, y: np.sin(np.pi * x) ** 2 * np.sin(np.pi * y) ** 2 * np.cos(np.pi * t) / np.pi  # noqa: E731
    a = -(psi(x, y + dy / 2) - psi(x, y - dy / 2)) / dy
    b = (psi(x + dx / 2, y) - psi(x - dx / 2, y)) / dx
    return a, b


def _fine_trace(x, y, t, tau, dx, dy, n=2000):
    """The same characteristic integrated back with n small RK4 steps."""
    h = -tau / n
    s = t + tau
    for _ in range(n):
        a1, b1 = _vel(x, y, s, dx, dy)
        a2, b2 = _vel(x + h / 2 * a1, y + h / 2 * b1, s + h / 2, dx, dy)
        a3, b3 = _vel(x + h / 2 * a2, y + h / 2 * b2, s + h / 2, dx, dy)
        a4, b4 = _vel(x + h * a3, y + h * b3, s + h, dx, dy)
        x, y = x + h / 6 * (a1 + 2 * a2 + 2 * a3 + a4), y + h / 6 * (b1 + 2 * b2 + 2 * b3 + b4)
        s += h
    return x, y


def test_foot_is_a_fourth_order_trace_back():
    """The oracle's one-step foot agrees with a fine integration of the same
    characteristic to O(tau^5): a wrong stage, sign or time offset fails."""
    dx = dy = 1.0 / 64
    rng = np.random.default_rng(5)
    for _ in range(6):
        x, y, t = rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0, 1)
        for tau in (0.004, 0.008):
            fx, fy = oracle.swirl_foot(x, y, t, tau, dx, dy)
            gx, gy = _fine_trace(x, y, t, tau, dx, dy)
            assert abs(fx - gx) + abs(fy - gy) <= 50 * tau ** 5, (x, y, t, tau)
            # a trace in the wrong direction would be off by about 2 |v| tau
            assert abs(fx - x) + abs(fy - y) > 100 * (abs(fx - gx) + abs(fy - gy)) or abs(fx - x) + abs(fy - y) < 1e-12


def test_constant_state_uniform():
    """Theorem of Sec. 4.3: the face-midpoint fluxes are differences of Psi at
    cell corners, so a constant state is kept on a Cartesian grid."""
    N = 32
    d0 = {k: np.full((1, N, N), 1.0) for k in KINDS}
    d0["dx"] = d0["dy"] = 1.0 / N
    out = oracle.run_periodic_swirl(d0, 0.6 / N, 20, t0=0.1)
    for k in KINDS:
        assert np.abs(out[k] - 1.0).max() <= 1e-14, k


def _diag_hier(nsteps, subcycle, n0=2):
    m, lc = 8, 1
    h = oracle.Hier(3, m, n0, n0, lc + 1)
    h.set_leaves(afsynth.diagonal_leaves(n0, lc))
    h.init_from(afsynth.polynomial([{(0, 0): 1.0}]), nq=2)
    dt0 = 0.6 * h.dx(0)
    if subcycle:
        h.run(dt0, nsteps)
    else:
        h.run_global(0.5 * dt0, 2 * nsteps)  # the step of the finer level everywhere
    err = 0.0
    for k in range(len(h.leaves())):
        err = max(err, float(np.abs(h.get_block(k)["avg"][0, 2:2 + m, 2:2 + m] - 1.0).max()))
    return err, h.time, dt0


def test_constant_state_amr_without_subcycling():
    """Corollary of Sec. 4.3: with global time stepping the summed fine
    fluxes equal the coarse flux of a constant state, which is kept to
    round-off (a few ulps after 16 steps)."""
    err, t, dt0 = _diag_hier(8, subcycle=False)
    assert abs(t - 8 * dt0) < 1e-15
    print("swirl constant state, global steps:", err)
    assert err <= 5e-15


def test_constant_state_amr_with_subcycling_is_fourth_order_in_dt():
    """With subcycling the coarse cell at a coarse-fine face sees one Simpson
    rule in time on its coarse faces and the composite rule of the two fine
    substeps on the fine face (Sec. 4.3: "components at the intermediate time
    that are in general not balanced").  The imbalance is the difference of
    the two quadratures, O(dt^4) per step: halving the mesh divides it by
    about 16."""
    e1, _, _ = _diag_hier(8, subcycle=True, n0=2)
    e2, _, _ = _diag_hier(8, subcycle=True, n0=4)
    print("swirl constant state, subcycling:", e1, e2, e1 / e2)
    assert e1 > 1e-13 and 12.0 <= e1 / e2 <= 20.0


def test_conservation():
    N = 32
    d0 = afsynth.dofs_periodic(afsynth.swirl_gaussians(), N, N, nq=4)
    out = oracle.run_periodic_swirl(d0, 0.6 / N, 16)
    assert abs(out["avg"].sum() - d0["avg"].sum()) <= 1e-14 * np.abs(d0["avg"]).sum()


def test_third_order_at_return_time():
    """At t = 1 the field has reversed and the exact solution is the initial
    data (eq. id_swirl): EOC 32 -> 64 near 3."""
    data = afsynth.swirl_gaussians()
    errs = []
    for N in (32, 64):
        d0 = afsynth.dofs_periodic(data, N, N, nq=4)
        n = int(np.ceil(1.0 / (0.6 / N)))
        out = oracle.run_periodic_swirl(d0, 1.0 / n, n)
        errs.append(np.abs(out["avg"] - d0["avg"]).sum() / N ** 2)
    eoc = np.log2(errs[0] / errs[1])
    print("swirl L1", errs, "EOC", eoc)
    assert 2.6 <= eoc <= 3.4
