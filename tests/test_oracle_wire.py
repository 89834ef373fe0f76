"""Pins of the oracle's wire boundary conditions (periodic z, isolated x and
y; Sec. II.C lists the wire BC): cell averages against adaptive quadrature,
FFT convolution against the dense sum, positive definiteness, and two closed
forms (a z-modulated Gaussian through its Hankel transform, and a Gaussian
line charge)."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import exp1, j0, k0

from oracle import green, pcg, wire
from oracle.dense import dense_solve


def test_off_origin_cell_averages_match_adaptive_quadrature():
    h, rw = 0.4, 20.0
    for kz in (0.0, 1.3, 7.0):
        for mx, my in ((1, 0), (1, 1), (3, 2), (0, 5)):
            got = wire.cell_average(mx, my, kz, h, rw)
            f = lambda y, x: (-2 * np.log(np.hypot(x, y) / rw) if kz == 0.0
                              else 2 * k0(kz * np.hypot(x, y)))
            ref, _ = integrate.dblquad(f, (mx - 0.5) * h, (mx + 0.5) * h,
                                       (my - 0.5) * h, (my + 0.5) * h, epsabs=0, epsrel=1e-12)
            assert abs(got / (ref / h ** 2) - 1) < 5e-9, (kz, mx, my)   # 10-point rule


@pytest.mark.parametrize("kz", [0.0, 0.5, 3.0, 7.8])
def test_origin_cell_average_matches_adaptive_polar_quadrature(kz):
    h, rw = 0.4, 20.0
    got = wire.cell_average(0, 0, kz, h, rw)
    g = (lambda r: -2 * np.log(r / rw)) if kz == 0.0 else (lambda r: 2 * k0(kz * r))
    inner = lambda t: integrate.quad(lambda r: g(r) * r, 0, h / (2 * np.cos(t)),
                                     epsabs=0, epsrel=1e-13, limit=200)[0]
    ref = 8 / h ** 2 * integrate.quad(inner, 0, np.pi / 4, epsabs=0, epsrel=1e-13)[0]
    assert abs(got / ref - 1) < 1e-11


@pytest.mark.parametrize("shape,h", [((4, 5, 6), 0.4), ((6, 4, 3), 0.7), ((3, 7, 5), 0.3)])
def test_fft_equals_dense_and_positive_definite(shape, h):
    rng = np.random.default_rng(4)
    f = rng.normal(size=shape)
    u = green.VacuumSolver(shape, h, "wire").apply(f)
    G = green.dense_green(shape, h, "wire")
    assert np.abs(u - (G @ f.ravel()).reshape(shape)).max() <= 1e-13 * np.abs(u).max()
    assert np.allclose(G, G.T, rtol=0, atol=1e-14 * np.abs(G).max())
    assert np.linalg.eigvalsh(G).min() > 0.0


def _centre_axis(n, h):
    return (np.arange(n) - (n - 1) / 2.0) * h


def test_modulated_gaussian_closed_form():
    # f = cos(kz z) exp(-rho^2 / 2 s^2) / (2 pi s^2): u = cos(kz z) U(rho) with
    # U(rho) = 2 int_0^inf J0(q rho) exp(-q^2 s^2/2) q / (q^2 + kz^2) dq
    s, lz = 0.8, 2.0
    errs = []
    for n, h in ((41, 0.25), (61, 1.0 / 6.0)):
        nz = int(round(lz / h))
        x = _centre_axis(n, h)
        z = np.arange(nz) * h
        kz = 2 * np.pi / lz
        rho2 = x[None, :] ** 2 + x[:, None] ** 2
        f = np.cos(kz * z)[:, None, None] * (np.exp(-rho2 / (2 * s * s)) / (2 * np.pi * s * s))[None]
        u = green.VacuumSolver((nz, n, n), h, "wire").apply(f)
        c = n // 2
        radii = [0, 1, 2, 4, 7, 12]
        got = np.array([u[0, c, c + m] for m in radii])
        ref = np.array([2 * integrate.quad(lambda q: j0(q * m * h) * np.exp(-q * q * s * s / 2)
                                           * q / (q * q + kz * kz), 0, np.inf, limit=400)[0]
                        for m in radii])
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    # second order: (1/6 / 1/4)^2 = 0.44
    assert errs[1] < 4e-3 and errs[1] < 0.6 * errs[0], errs


def test_gaussian_line_charge_closed_form():
    # uniform in z: u(rho) = -2 ln rho - E1(rho^2 / 2 s^2) + C; the kz = 0
    # kernel -2 ln(rho / Rw) fixes C = 2 ln Rw
    s, nz = 0.8, 4
    errs = []
    for n, h in ((41, 0.25), (61, 1.0 / 6.0)):
        x = _centre_axis(n, h)
        rho2 = x[None, :] ** 2 + x[:, None] ** 2
        f = np.broadcast_to(np.exp(-rho2 / (2 * s * s)) / (2 * np.pi * s * s), (nz, n, n))
        u = green.VacuumSolver((nz, n, n), h, "wire").apply(np.ascontiguousarray(f))
        c = n // 2
        rw = wire.wire_radius(n, n, h)
        ref = lambda r: (2 * np.log(rw) + np.euler_gamma - np.log(2 * s * s) if r == 0 else
                         2 * np.log(rw) - 2 * np.log(r) - exp1(r * r / (2 * s * s)))
        radii = [0, 1, 3, 6, 10]
        got = np.array([u[1, c, c + m] for m in radii])
        want = np.array([ref(m * h) for m in radii])
        errs.append(np.abs(got - want).max() / np.abs(want).max())
    assert errs[1] < 1e-3 and errs[1] < 0.6 * errs[0], errs


def test_pcg_matches_dense_solve_wire():
    from paper_1509_00680_amd import workloads as W
    shape, h = (4, 5, 6), 0.5
    rng = np.random.default_rng(9)
    eps = 1.0 + 20.0 * rng.random(shape)
    rho = rng.normal(size=shape)
    res = pcg.pcg_solve(rho, eps, h, "wire", tol=1e-12)
    assert res.converged
    ref = dense_solve(rho, eps, h, "wire")
    assert np.abs(res.phi - ref).max() <= 1e-9 * np.abs(ref).max()
