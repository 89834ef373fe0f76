"""Pins of the oracle's rigid cavity (Eq. RigCav, analytic q of Eq. corr) and
polarization charge (Eqs. rhoiter, remap, rhopol)."""
import numpy as np
import pytest

from oracle import cavity, stencil
from oracle.pcg import pcg_solve
from paper_1509_00680_amd import workloads as W


def test_first_weights_textbook_values():
    assert np.allclose(cavity.fd_first_derivative_weights(1), [0.5], atol=1e-16)
    assert np.allclose(cavity.fd_first_derivative_weights(2), [2 / 3, -1 / 12], atol=1e-16)
    assert np.allclose(cavity.fd_first_derivative_weights(3), [3 / 4, -3 / 20, 1 / 60],
                       atol=1e-16)


@pytest.mark.parametrize("M", [1, 4, 8])
def test_first_difference_order(M):
    # exact on polynomials of degree 2M, not on degree 2M + 1
    n, h = 2 * M + 12, 0.4
    x = (np.arange(n) - n / 2) * h
    inner = slice(M, n - M)
    rng = np.random.default_rng(10 + M)
    for deg, exact in ((2 * M, True), (2 * M + 1, False)):
        coef = rng.normal(size=deg + 1)
        coef[0] = 1.0
        f = np.polyval(coef, x)
        d1 = np.polyval(np.polyder(coef), x)
        got = cavity.first_difference(f[None, None, :], 2, h, M, periodic=False)[0, 0]
        err = np.max(np.abs(got[inner] - d1[inner])) / np.max(np.abs(d1[inner]))
        if exact:
            assert err < 1e-10, (deg, err)
        else:
            assert err > 1e-10, (deg, err)


def test_first_difference_periodic_wrap():
    # exact for a trigonometric polynomial well below the Nyquist frequency only
    # up to the order's error; the wrap itself: shifting f shifts f'
    n, h = 40, 0.3
    rng = np.random.default_rng(3)
    f = rng.normal(size=(1, 1, n))
    d = cavity.first_difference(f, 2, h, 8, periodic=True)
    d_shift = cavity.first_difference(np.roll(f, 7, axis=2), 2, h, 8, periodic=True)
    assert np.allclose(np.roll(d, 7, axis=2), d_shift, rtol=0, atol=1e-13)


def test_one_atom_is_the_sphere_cavity():
    shape, h = (20, 22, 24), 0.4
    eps, _ = cavity.rigid_cavity(shape, h, [[0.0, 0.0, 0.0, 2.5]], 0.4, W.EPS_WATER)
    ref = W.sphere_cavity(shape, h, 2.5, 0.4, W.EPS_WATER)
    assert np.max(np.abs(eps - ref)) < 1e-12 * W.EPS_WATER


def test_cavity_limits():
    shape, h = (30, 30, 30), 0.4
    atoms = [[-1.0, 0.0, 0.0, 2.0], [1.2, 0.3, -0.2, 2.2]]
    eps, q = cavity.rigid_cavity(shape, h, atoms, 0.3, 80.0)
    assert eps.min() >= 1.0 and eps.max() <= 80.0
    assert eps.max() > 79.999                 # the corners are solvent
    x = (np.arange(30) - 14.5) * h
    i = np.argmin(np.abs(x + 1.0))
    assert eps[15, 15, i] < 1.0 + 1e-6          # inside the first atom
    assert np.all(np.isfinite(q))


def test_analytic_q_matches_order16_differences():
    # q from the product rule against q = sqrt(eps) lap_h sqrt(eps) of the
    # (separately pinned) order-16 stencil.  Radii of 4.5-5 Delta, as for
    # physical cavities.  The difference is discretization error: it falls by
    # more than 5x from h = 0.15 to h = 0.1 and is below 1e-3 of max|q| there,
    # while dropping the cross terms, flipping the sign of the gradient term
    # or halving 2 h'/r changes q by 17% to 150% of max|q|.
    atoms = [[0.4, -0.3, 0.2, 2.0], [-0.7, 0.5, -0.1, 1.8], [0.1, 0.6, 0.6, 2.1]]
    errs = []
    for n, h in ((64, 0.15), (96, 0.1)):
        eps, q = cavity.rigid_cavity((n, n, n), h, atoms, 0.4, 30.0)
        qfd = stencil.q_field(eps, h, "free", 16)
        inner = (slice(8, n - 8),) * 3
        errs.append(np.max(np.abs(q[inner] - qfd[inner])) / np.max(np.abs(q)))
    assert errs[1] < 1e-3 and errs[1] < errs[0] / 5, errs


def test_atom_on_a_grid_point_reading():
    # r = 0 on a grid point: gradient 0 and Laplacian h''(0), so that
    # q(0) = (eps0 - 1) h''(0) / 2 with h''(0) = -2 t h'(0) / Delta, t = -d/Delta
    h, d, delta, eps0 = 0.5, 2.0, 0.4, 10.0
    eps, q = cavity.rigid_cavity((9, 9, 9), h, [[0.0, 0.0, 0.0, d]], delta, eps0)
    t = -d / delta
    h1 = np.exp(-t * t) / (delta * np.sqrt(np.pi))
    expect = 0.5 * (eps0 - 1.0) * (-2.0 * t / delta * h1)
    assert np.isfinite(q).all() and abs(eps[4, 4, 4] - 1.0) < 1e-10
    assert abs(q[4, 4, 4] - expect) < 1e-12 * abs(expect)


def test_periodic_minimum_image():
    shape, h = (16, 16, 16), 0.5
    L = 16 * h
    a = [[3.9, 0.2, -0.1, 1.5]]
    b = [[3.9 - L, 0.2, -0.1 + L, 1.5]]
    e1, q1 = cavity.rigid_cavity(shape, h, a, 0.4, 20.0, bc="periodic")
    e2, q2 = cavity.rigid_cavity(shape, h, b, 0.4, 20.0, bc="periodic")
    assert np.allclose(e1, e2, rtol=0, atol=1e-12) and np.allclose(q1, q2, rtol=0, atol=1e-10)
    # surface: z is not wrapped
    e3, _ = cavity.rigid_cavity(shape, h, b, 0.4, 20.0, bc="surface")
    assert np.max(np.abs(e3 - e1)) > 1.0


def test_polarization_charge_manufactured():
    # analytic rho_pol = -lap(phi)/(4 pi) - rho for the manufactured Gaussian
    # phi in an erf cavity: the order-16 form converges to it (the difference
    # falls by more than 20x from h = 1/8 to h = 1/12 and is 1e-5 there),
    # while the printed sign of the (1 - 1/eps) rho term is off by O(1)
    errs = []
    for n in (64, 96):
        sigma = 0.8
        prob, phi = W.manufactured_gaussian(n, box=8.0, sigma=sigma, d0=2.5, delta=0.6)
        x, y, z = W.grid_coords(prob.shape, prob.h)
        r2 = x * x + y * y + z * z
        s2 = sigma * sigma
        lap = (r2 / (s2 * s2) - 3.0 / s2) * phi
        ref = -lap / (4 * np.pi) - prob.rho
        got = cavity.polarization_charge(prob.rho, prob.eps, phi, prob.h, "free", 16)
        errs.append(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert errs[1] < 1e-5 and errs[1] < errs[0] / 20, errs
    flipped = got + 2 * (1 - 1 / prob.eps) * prob.rho
    assert np.max(np.abs(flipped - ref)) / np.max(np.abs(ref)) > 0.5


def test_polarization_charge_gauss_law():
    # a unit charge in a spherical cavity: the solvent's total bound charge is
    # -(1 - 1/eps0) Q (Gauss's law with D = Q/(4 pi r^2) outside the cavity)
    # (discretization: 7.6e-4 at h = 0.18 against Delta = 0.6)
    prob = W.single_sphere(n=64, h=0.18, sigma=0.6, q=1.0, d0=2.5, delta=0.6)
    res = pcg_solve(prob.rho, prob.eps, prob.h, prob.bc, tol=1e-9)
    assert res.converged
    pol = cavity.polarization_charge(prob.rho, prob.eps, res.phi, prob.h, prob.bc, 16)
    total = float(np.sum(pol)) * prob.h ** 3
    q = float(np.sum(prob.rho)) * prob.h ** 3
    expect = -(1.0 - 1.0 / W.EPS_WATER) * q
    assert abs(total - expect) < 2e-3 * abs(expect), (total, expect)
