"""Oracle pins for Burgers' equation (Sec. 2.2 and Sec. 4.4):
q_t + (q^2/2)_x + (q^2/2)_y = 0. Point values come from fixed-point
iterations of q(P, t+tau) = q^n(P - q tau (1, 1)) (eq. burgers-sol,
eq. Burgers-iterativ), starting from the mean of the neighbouring cell
averages. Fluxes are the Simpson rule of q^2/2."""
import math

import numpy as np
import pytest

import afsynth
import oracle

KINDS = ("avg", "corner", "xedge", "yedge")
G = 2


def _cell_dofs(blk, i, j):
    """The 9 DOFs of cell (i, j) of a block, in the order of recon_eval:
    average, corners (ll, rl, lu, ru), edges (left, right, bottom, top)."""
    a = lambda k, ii, jj: blk[k][0, jj + G, ii + G]  # noqa: E731
    return np.array([a("avg", i, j), a("corner", i, j), a("corner", i + 1, j), a("corner", i, j + 1),
                     a("corner", i + 1, j + 1), a("xedge", i, j), a("xedge", i + 1, j), a("yedge", i, j),
                     a("yedge", i, j + 1)])


def _node(kind, i, j):
    # node position in cell units (cell k spans [k - 1/2, k + 1/2])
    return (i - 0.5 if kind != "yedge" else float(i)), (j - 0.5 if kind != "xedge" else float(j))


def _guess(blk, kind, i, j):
    """Starting speed of Sec. 2.2: the mean of the averages around the node."""
    a = lambda ii, jj: blk["avg"][0, jj + G, ii + G]  # noqa: E731
    if kind == "corner":
        return 0.25 * (a(i - 1, j) + a(i, j) + a(i - 1, j - 1) + a(i, j - 1))
    if kind == "xedge":
        return 0.5 * (a(i - 1, j) + a(i, j))
    return 0.5 * (a(i, j) + a(i, j - 1))


def _eval_at(blk, X, Y):
    """q^n at cell-unit position (X, Y): the reconstruction of the cell that
    contains it (positions here never lie on a face)."""
    ci, cj = int(math.floor(X + 0.5)), int(math.floor(Y + 0.5))
    v = oracle.recon_eval(_cell_dofs(blk, ci, cj), np.array([2.0 * (X - ci)]), np.array([2.0 * (Y - cj)]))
    return float(v[0])


def _random_block(m, seed):
    """Smooth-ish random data: a sum of a few low modes plus a constant, so
    that the reconstruction stays near the data range."""
    rng = np.random.default_rng(seed)
    terms = {(0, 0): 0.4}
    for p in range(3):
        for q in range(3 - p):
            if p + q:
                terms[(p, q)] = rng.uniform(-0.3, 0.3)
    data = afsynth.polynomial([terms])
    return afsynth.dofs_block(data, 8, G, -0.2, 0.1, 0.05, 0.05, 4)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_one_iteration_is_the_reconstruction_at_the_guess_foot(seed):
    """With one iteration the new point value is q^n at P - Q0 dt (1, 1), Q0
    the mean of the neighbouring averages: checked node by node against the
    reconstruction evaluated directly (pins the starting guess, the sign and
    the direction of the displacement)."""
    m, dx = 8, 0.05
    blk = _random_block(m, seed)
    dt = 0.3 * dx
    out = oracle.patch_step_burgers(m, blk, dx, dx, dt, iters=1)
    for kind in ("corner", "xedge", "yedge"):
        for (i, j) in [(0, 0), (3, 5), (7, 2), (4, 4), (1, 7)]:
            Q0 = _guess(blk, kind, i, j)
            X, Y = _node(kind, i, j)
            want = _eval_at(blk, X - Q0 * dt / dx, Y - Q0 * dt / dx)
            assert abs(out[kind][0, j + G, i + G] - want) <= 1e-14, (kind, i, j)


def test_iterations_on_affine_data():
    """q0 = alpha + beta (x + y): the reconstruction is exact and the mean of
    the neighbouring averages is the node value A, so k iterations give the
    fixed-point map Q <- A - 2 beta tau Q applied k times to A; many
    iterations converge to the exact solution A / (1 + 2 beta tau) of eq.
    burgers-sol."""
    m, dx, alpha, beta = 8, 0.05, 0.3, 0.5
    data = afsynth.polynomial([{(0, 0): alpha, (1, 0): beta, (0, 1): beta}])
    x0p, y0p = -0.2, 0.1
    blk = afsynth.dofs_block(data, m, G, x0p, y0p, dx, dx, 4)
    dt = 0.4 * dx
    for iters in (1, 2, 3, 40):
        out = oracle.patch_step_burgers(m, blk, dx, dx, dt, iters=iters)
        for kind in ("corner", "xedge", "yedge"):
            for (i, j) in [(0, 0), (5, 3), (8, 8) if kind == "corner" else (2, 6)]:
                X, Y = _node(kind, i, j)
                s = x0p + (X + 0.5) * dx + y0p + (Y + 0.5) * dx
                A = alpha + beta * s
                Q = A
                for _ in range(iters):
                    Q = A - 2 * beta * dt * Q
                assert abs(out[kind][0, j + G, i + G] - Q) <= 1e-14, (iters, kind, i, j)
                if iters == 40:
                    assert abs(Q - A / (1 + 2 * beta * dt)) <= 1e-15


def test_two_iterations_are_the_method():
    """The default patch step is the two-iteration one."""
    m, dx = 8, 0.05
    blk = _random_block(m, 7)
    a = oracle.patch_step(4, m, blk, dx, dx, 0.3 * dx)
    b = oracle.patch_step_burgers(m, blk, dx, dx, 0.3 * dx, iters=2)
    for k in KINDS:
        np.testing.assert_array_equal(a[k], b[k])


def test_constant_state_is_kept():
    N = 16
    d0 = {k: np.full((1, N, N), 0.7) for k in KINDS}
    d0["dx"] = d0["dy"] = 1.0 / N
    out = oracle.run_periodic(4, d0, 0.5 / N / 0.7, 12)
    for k in KINDS:
        assert np.abs(out[k] - 0.7).max() <= 1e-15, k


def _periodic(N, nq=4):
    return afsynth.dofs_periodic(afsynth.burgers_sinsin(), N, N, nq=nq)


def test_conservation_before_and_after_the_shock():
    """The sum of the averages is kept to round-off, also past the shock time
    1 / (2 pi) where the unlimited method oscillates."""
    N = 32
    d0 = _periodic(N)
    dt = 0.5 / N / 1.1
    out = oracle.run_periodic(4, d0, dt, int(0.3 / dt))
    s0, s1 = d0["avg"].sum(), out["avg"].sum()
    assert abs(s1 - s0) <= 1e-13 * np.abs(d0["avg"]).sum()


def _l1_error(avg, N, T):
    ex = afsynth.InitialData(1, lambda x, y: afsynth.burgers_sinsin().exact(x, y, T))
    ref = afsynth.dofs_periodic(ex, N, N, nq=4)["avg"][0]
    return float(np.abs(avg - ref).sum()) / N ** 2


def test_third_order_before_the_shock():
    """Sec. 4.4: eq. sinsin01 to t = 0.05 at CFL 0.5 (largest |q| = 1.1);
    L1 error of the averages against the exact implicit solution, EOC near
    3."""
    T, errs = 0.05, []
    for N in (32, 64, 128):
        n = math.ceil(T / (0.5 / N / 1.1))
        out = oracle.run_periodic(4, _periodic(N), T / n, n)
        errs.append(_l1_error(out["avg"][0], N, T))
    eoc = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    print("burgers L1", errs, "EOC", eoc)
    assert 2.6 <= eoc[1] <= 3.4, eoc


def test_amr_antidiagonal_third_order_and_conservation():
    """Sec. 4.4: refinement forced along the diagonal from the upper-left to
    the lower-right patch, subcycling and the conservative fix; EOC near 3
    over two resolutions, and the sum of the averages kept."""
    T, m, errs = 0.05, 8, []
    for n0 in (4, 8):
        h = oracle.Hier(4, m, n0, n0, 1)
        leaves = afsynth.antidiagonal_leaves(n0, 0)
        h.set_leaves(leaves)
        h.init_from(afsynth.burgers_sinsin(), nq=4)
        h.fill()
        s0 = h.total()
        n = math.ceil(T / (0.5 * h.dx(0) / 1.1))
        h.run(T / n, n)
        s1 = h.total()
        assert abs(s1 - s0).max() <= 1e-13
        ex = afsynth.InitialData(1, lambda x, y: afsynth.burgers_sinsin().exact(x, y, T))
        err = 0.0
        for k, (l, ix, iy) in enumerate(leaves):
            dx = h.dx(l)
            ref = afsynth.dofs_block(ex, m, G, ix * m * dx, iy * m * dx, dx, dx, 4)["avg"][0, G:G + m, G:G + m]
            err += float(np.abs(h.get_block(k)["avg"][0, G:G + m, G:G + m] - ref).sum()) * dx * dx
        errs.append(err)
    eoc = math.log2(errs[0] / errs[1])
    print("burgers AMR L1", errs, "EOC", eoc)
    assert 2.5 <= eoc <= 3.5, eoc
