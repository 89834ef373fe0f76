"""Pins of the oracle's vacuum Poisson solver (Eq. SPe; Sec. II.C) against
closed forms, brute force and sum rules that do not reuse its code paths."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf, erfc

from oracle import green
from paper_1509_00680_amd import workloads as W


def test_cube_integral_origin_closed_form():
    # integral of 1/r over the unit cube centred at 0 is 3 ln(2 + sqrt 3) - pi/2
    exact = 3.0 * math.log(2.0 + math.sqrt(3.0)) - math.pi / 2.0
    assert abs(green.cube_integral_exact(0, 0, 0) - exact) < 1e-14


@pytest.mark.parametrize("m", [(1, 0, 0), (2, 1, 0), (3, 2, 1), (1, 1, 1)])
def test_cube_integral_quadrature(m):
    val, _ = integrate.tplquad(
        lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z),
        m[0] - 0.5, m[0] + 0.5, m[1] - 0.5, m[1] + 0.5, m[2] - 0.5, m[2] + 0.5,
        epsabs=1e-13, epsrel=1e-13)
    assert abs(green.cube_integral_exact(*m) - val) < 1e-11


@pytest.mark.parametrize("a", [1, 3, 8, 13])
def test_cube_integral_additivity(a):
    # the (2a+1)^3 unit cubes tile a cube of side 2a+1, and the integral of
    # 1/r over a cube of side s is s^2 I(0); a = 13 mixes exact and expansion.
    m = np.arange(-a, a + 1)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    total = green.cell_averaged_inverse_distance(mx, my, mz).sum()
    expect = (2 * a + 1) ** 2 * green.cube_integral_exact(0, 0, 0)
    tol = 1e-13 if a <= green.NEAR_CUTOFF else 1e-11
    assert abs(total / expect - 1.0) < tol


def test_far_expansion_matches_exact_beyond_cutoff():
    for m in [(9, 0, 0), (9, 9, 9), (9, 4, 2), (12, 1, 0)]:
        e = green.cube_integral_exact(*m)
        f = green.cube_integral_far(*m)
        assert abs(f / e - 1.0) < 5e-11


@pytest.mark.parametrize("bc,shape", [("free", (5, 7, 9)), ("free", (4, 4, 4)),
                                      ("periodic", (5, 6, 4)), ("surface", (5, 6, 4)),
                                      ("surface", (3, 4, 6))])
def test_fft_convolution_equals_dense(bc, shape):
    rng = np.random.default_rng(7)
    f = rng.normal(size=shape)
    solver = green.VacuumSolver(shape, 0.45, bc)
    g = green.dense_green(shape, 0.45, bc)
    u_dense = (g @ f.ravel()).reshape(shape)
    assert np.abs(solver.apply(f) - u_dense).max() < 1e-13 * np.abs(u_dense).max() * 10


@pytest.mark.parametrize("bc", ["free", "surface"])
def test_dense_green_positive_definite(bc):
    g = green.dense_green((4, 5, 6), 0.5, bc)
    assert np.allclose(g, g.T, atol=1e-14)
    assert np.linalg.eigvalsh(g).min() > 0.0


def test_surface_unshifted_kernel_is_indefinite():
    # -2 pi |z| alone gives one negative eigenvalue (why the shift exists)
    g = green.dense_green_surface((6, 4, 4), 0.5, k0_offset=0.0)
    ev = np.linalg.eigvalsh(g)
    assert ev[0] < 0.0 < ev[1]


def _vacuum_energy(n, h, sigma=1.0, q=1.0):
    shape = (n, n, n)
    rho = W.gaussian_sum(shape, h, [(0, 0, 0)], [sigma], [q])
    u = green.VacuumSolver(shape, h, "free").apply(rho)
    return 0.5 * h ** 3 * float(np.sum(rho * u))


def test_free_gaussian_energy_second_order():
    # E = q^2/(2 sqrt(pi) sigma); cell averaging gives E_h = E - (pi h^2/12) int rho^2
    # + O(h^4) with int rho^2 = q^2 / (8 pi^1.5 sigma^3)
    sigma = 1.0
    E = 1.0 / (2.0 * math.sqrt(math.pi) * sigma)
    irho2 = 1.0 / (8.0 * math.pi ** 1.5 * sigma ** 3)
    rem = []
    for n, h in [(48, 0.35), (96, 0.175)]:
        Eh = _vacuum_energy(n, h, sigma)
        rem.append(Eh - (E - math.pi * h * h / 12.0 * irho2))
    assert abs(rem[0]) < 3e-5
    assert 10.0 < rem[0] / rem[1] < 22.0        # fourth-order remainder


def test_free_gaussian_potential_pointwise():
    n, h, sigma = 48, 0.35, 1.0
    shape = (n, n, n)
    rho = W.gaussian_sum(shape, h, [(0, 0, 0)], [sigma], [1.0])
    u = green.VacuumSolver(shape, h, "free").apply(rho)
    x, y, z = W.grid_coords(shape, h)
    r = np.sqrt(x * x + y * y + z * z)
    phi = erf(r / (math.sqrt(2) * sigma)) / r
    corrected = phi - math.pi * h * h / 6.0 * rho
    assert np.abs(u - corrected).max() < 3e-4
    assert np.abs(u - phi).max() > 3e-3       # the h^2 term is really there


def test_periodic_cosine_exact():
    shape = (8, 6, 10)
    h = 0.4
    x, y, z = W.grid_coords(shape, h)
    kx, kz = 2 * math.pi / (10 * h), 2 * math.pi * 2 / (8 * h)
    f = np.cos(kx * x) * np.cos(kz * z) * np.ones(shape)
    u = green.VacuumSolver(shape, h, "periodic").apply(f)
    assert np.abs(u - 4 * math.pi / (kx * kx + kz * kz) * f).max() < 1e-12


def _surface_sheet_error(nz, h, sigma=0.8):
    nxy = 8
    shape = (nz, 1, nxy)
    x, _, z = W.grid_coords(shape, h)
    k = 2 * math.pi / (nxy * h)
    gz = np.exp(-z * z / (2 * sigma ** 2)) / math.sqrt(2 * math.pi * sigma ** 2)
    f = np.cos(k * x) * gz
    u = green.VacuumSolver(shape, h, "surface").apply(f)
    c = 1.0 / (math.sqrt(2) * sigma)
    conv = 0.5 * math.exp(k * k * sigma * sigma / 2) * (
        np.exp(-k * z) * erfc((k * sigma ** 2 - z) * c)
        + np.exp(k * z) * erfc((k * sigma ** 2 + z) * c))
    exact = np.cos(k * x) * (2 * math.pi / k) * conv
    return np.abs(u - exact).max()


def test_surface_kpar_mode_closed_form():
    # cos(kx) times a normalized Gaussian sheet: potential (2 pi/k) e^{-k|z|} * g
    e1 = _surface_sheet_error(48, 0.25)
    e2 = _surface_sheet_error(96, 0.125)
    assert e1 < 2e-3
    assert e1 / e2 > 3.5                      # at least second order in h


def _surface_k0_error(nz, h, sigma=0.6, a=1.5):
    shape = (nz, 2, 2)
    _, _, z = W.grid_coords(shape, h)
    def g(t):
        return np.exp(-t * t / (2 * sigma ** 2)) / math.sqrt(2 * math.pi * sigma ** 2)
    f = (g(z - a) - g(z + a)) * np.ones(shape)
    u = green.VacuumSolver(shape, h, "surface").apply(f)
    def F(t):      # int |t - s| g(s) ds
        return t * erf(t / (math.sqrt(2) * sigma)) + math.sqrt(2 / math.pi) * sigma * np.exp(
            -t * t / (2 * sigma ** 2))
    exact = -2 * math.pi * (F(z - a) - F(z + a)) * np.ones(shape)
    return np.abs(u - exact).max()


def test_surface_k0_mode_closed_form():
    # neutral pair of sheets: -2 pi int |z - z'| f(z') dz' (the shift cancels)
    e1 = _surface_k0_error(40, 0.3)
    e2 = _surface_k0_error(80, 0.15)
    assert e1 < 0.05                         # |u| ~ 19 here
    assert 3.0 < e1 / e2 < 5.0
