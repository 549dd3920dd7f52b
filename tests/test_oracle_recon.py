"""Pins for the oracle's reconstruction (Sec. 2, eq. poly) and spherical
means (Sec. 2.3, eq. sphe-mean).  Each check compares against something the
mathematics fixes independently of the oracle's own formulas."""
import numpy as np
import pytest
from scipy import integrate

import oracle


def _biquad(c):
    return lambda x, y: sum(c[m, n] * x ** m * y ** n for m in range(3) for n in range(3))


def _mono_avg(k):  # mean of x^k over [-1,1]
    return 1.0 if k == 0 else (0.0 if k % 2 else 1.0 / (k + 1))


def _dofs(f, avg):
    return [avg, f(-1, -1), f(1, -1), f(-1, 1), f(1, 1), f(-1, 0), f(1, 0), f(0, -1), f(0, 1)]


@pytest.mark.parametrize("seed", range(5))
def test_reconstruction_reproduces_biquadratics(seed):
    """A biquadratic is fixed by its 8 boundary points and its average, so the
    reconstruction must return it exactly (closed-form moments of x^m y^n)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((3, 3))
    f = _biquad(c)
    avg = sum(c[m, n] * _mono_avg(m) * _mono_avg(n) for m in range(3) for n in range(3))
    xs, ys = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50)
    got = oracle.recon_eval(_dofs(f, avg), xs, ys)
    np.testing.assert_allclose(got, f(xs, ys), atol=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_reconstruction_average_and_interpolation(seed):
    """For arbitrary (non-polynomial) DOFs: the reconstruction interpolates the
    eight points and its average -- integrated by Gauss-Legendre quadrature,
    not by Simpson -- equals the given average."""
    rng = np.random.default_rng(100 + seed)
    d = rng.standard_normal(9)
    nodes = [(-1, -1), (1, -1), (-1, 1), (1, 1), (-1, 0), (1, 0), (0, -1), (0, 1)]
    got = oracle.recon_eval(d, [p[0] for p in nodes], [p[1] for p in nodes])
    np.testing.assert_allclose(got, d[1:], atol=1e-14)
    gx, gw = np.polynomial.legendre.leggauss(4)
    X, Y = np.meshgrid(gx, gx)
    W = np.outer(gw, gw)
    vals = oracle.recon_eval(d, X.ravel(), Y.ravel()).reshape(X.shape)
    assert abs((W * vals).sum() / 4.0 - d[0]) < 1e-13


def test_reconstruction_continuity_across_edge():
    """Two cells sharing an edge share its three nodes, so their
    reconstructions agree along the edge (continuous q^n, Sec. 2)."""
    rng = np.random.default_rng(7)
    left = rng.standard_normal(9)
    right = rng.standard_normal(9)
    # right cell's left nodes = left cell's right nodes
    right[1] = left[2]   # c_ll(right) = c_rl(left)
    right[3] = left[4]   # c_lu(right) = c_ru(left)
    right[5] = left[6]   # e_l(right) = e_r(left)
    eta = np.linspace(-1, 1, 17)
    a = oracle.recon_eval(left, np.ones_like(eta), eta)
    b = oracle.recon_eval(right, -np.ones_like(eta), eta)
    np.testing.assert_allclose(a, b, atol=1e-14)


def _num_sector_mean(m, n, quad, R):
    """Definition of the spherical mean restricted to one quadrant (eq.
    sphe-mean) by adaptive numerical quadrature after s = R sin(theta)."""
    lo = quad * np.pi / 2

    def integrand(theta, phi):
        s = R * np.sin(theta)
        return (s * np.cos(phi)) ** m * (s * np.sin(phi)) ** n * np.sin(theta)

    val, _ = integrate.dblquad(integrand, lo, lo + np.pi / 2, 0.0, np.pi / 2,
                               epsabs=1e-14, epsrel=1e-13)
    return val / (2 * np.pi)


@pytest.mark.parametrize("quad", range(4))
def test_sector_mean_matches_definition(quad):
    R = 0.37
    for m in range(4):
        for n in range(4 - m):
            coef = np.zeros((4, 4))
            coef[m, n] = 1.0
            got, rdm = oracle.sector_mean(coef, quad, R)
            ref = _num_sector_mean(m, n, quad, R)
            assert abs(got - ref) < 1e-12 * max(1.0, abs(ref)), (m, n, got, ref)
            # R d/dR by central differences of the numerical definition
            h = 1e-4
            fd = R * (_num_sector_mean(m, n, quad, R + h) - _num_sector_mean(m, n, quad, R - h)) / (2 * h)
            assert abs(rdm - fd) < 1e-7, (m, n, rdm, fd)


def test_full_disc_mean_of_constant_is_one():
    total = sum(oracle.sector_mean(np.eye(4)[0:1].T @ np.eye(4)[0:1], q, 0.5)[0] for q in range(4))
    assert abs(total - 1.0) < 1e-15
