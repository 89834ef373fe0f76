"""Pins of the oracle's finite differences and of q = sqrt(eps) lap sqrt(eps)
(Eq. corr; order-16 filters of Sec. II.C)."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import stencil
from paper_1509_00680_amd import workloads as W


def test_weights_textbook_values():
    assert np.allclose(stencil.fd_second_derivative_weights(1), [-2.0, 1.0], atol=1e-15)
    assert np.allclose(stencil.fd_second_derivative_weights(2), [-5 / 2, 4 / 3, -1 / 12],
                       atol=1e-15)
    assert np.allclose(stencil.fd_second_derivative_weights(3),
                       [-49 / 18, 3 / 2, -3 / 20, 1 / 90], atol=1e-15)


@pytest.mark.parametrize("M", [4, 8])
def test_weights_moment_conditions(M):
    # exactness on x^(2k): sum_j c_|j| j^(2k) = 2 for k = 1, 0 otherwise (k <= M)
    c = stencil.fd_second_derivative_weights(M)
    j = np.arange(1, M + 1, dtype=np.float64)
    for k in range(0, M + 1):
        mom = (c[0] if k == 0 else 0.0) + 2.0 * np.sum(c[1:] * j ** (2 * k))
        assert abs(mom - (2.0 if k == 1 else 0.0)) < 1e-9 * max(1.0, np.sum(np.abs(c[1:]) * j ** (2 * k)))


@pytest.mark.parametrize("M", [1, 3, 8])
def test_exact_on_polynomials(M):
    n, h = 3 * M + 8, 0.7
    x = (np.arange(n) - n / 2) * h
    rng = np.random.default_rng(M)
    coef = rng.normal(size=2 * M + 2)            # degree 2M+1
    f = np.polyval(coef, x)
    d2 = np.polyval(np.polyder(coef, 2), x)
    got = stencil.second_difference(f[None, None, :], 2, h, M, periodic=False)[0, 0]
    inner = slice(M, n - M)
    scale = np.abs(d2[inner]).max() + np.abs(f).max() / h ** 2 * 1e-12
    assert np.abs(got[inner] - d2[inner]).max() < 1e-9 * scale


def _radial_q(shape, h, d0, delta, eps0):
    x, y, z = W.grid_coords(shape, h)
    r = np.sqrt(x * x + y * y + z * z)
    u = (r - d0) / delta
    eps = 1 + (eps0 - 1) * 0.5 * (1 + erf(u))
    e1 = (eps0 - 1) * np.exp(-u * u) / (delta * math.sqrt(math.pi))
    e2 = -2 * u / delta * e1
    f = np.sqrt(eps)
    f1 = e1 / (2 * f)
    f2 = e2 / (2 * f) - e1 * e1 / (4 * eps * f)
    return eps, f * (f2 + 2 * f1 / r)


def test_q_matches_radial_analytic():
    # sphere cavity: q = sqrt(eps) (f'' + 2 f'/r), f = sqrt(eps); high order wins
    # (box 12.8 so that eps is flat at the faces and the ghosts are exact)
    shape, h = (64, 64, 64), 0.2
    eps, q_exact = _radial_q(shape, h, 3.0, 0.5, W.EPS_WATER)
    err = {o: np.abs(stencil.q_field(eps, h, "free", o) - q_exact).max() for o in (2, 8, 16)}
    scale = np.abs(q_exact).max()
    assert err[16] < 1e-3 * scale
    assert err[16] < err[8] < err[2]
    eps2, q2 = _radial_q((96, 96, 96), 12.8 / 96, 3.0, 0.5, W.EPS_WATER)
    err2 = np.abs(stencil.q_field(eps2, 12.8 / 96, "free", 16) - q2).max()
    assert err[16] / err2 > 8.0          # high order: (3/2)^p with p > 5


def test_q_periodic_spectral_exact():
    shape, h = (8, 10, 12), 0.5
    x, y, z = W.grid_coords(shape, h)
    k = 2 * math.pi / (12 * h)
    s = 2.0 + 0.5 * np.cos(k * x) * np.ones(shape)
    q = stencil.q_field(s * s, h, "periodic")
    assert np.abs(q - s * (-k * k * 0.5 * np.cos(k * x))).max() < 1e-12


def test_q_vanishes_for_constant_eps():
    for bc in ("free", "surface", "periodic"):
        q = stencil.q_field(np.full((6, 7, 8), 5.0), 0.3, bc)
        assert np.abs(q).max() < 1e-10
