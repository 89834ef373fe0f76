"""Finite differences and the fixed correction vector q (test infrastructure only).

Sec. II.B, Eq. corr: with the preconditioner of Eq. PCGdef the generalized
Poisson operator applied to a preconditioned residual reduces to
A v = -q v - 4 pi r, where q = sqrt(eps) lap sqrt(eps) is computed once per
dielectric function and kept fixed.  Sec. II.C states that order-16 central
finite-difference filters are used for derivatives (only Algorithm SC needs
them per iteration; for PCG they only enter q).

The order-2M central second difference has weights
  c_j = 2 (-1)^(j+1) (M!)^2 / (j^2 (M-j)! (M+j)!),  j = 1..M,
  c_0 = -2 sum_j c_j,
which follow from requiring exactness on polynomials of degree <= 2M+1.
Ghost values: replicate the edge value along free axes, wrap along periodic
axes.  With fully periodic boundaries q uses the spectral Laplacian, so that
the discrete operator annihilates constants exactly.
"""
from math import factorial

import numpy as np
from scipy import fft as sfft

from . import BC_FREE, BC_SURFACE, BC_PERIODIC, BC_WIRE
from .green import wavenumbers, rwavenumbers


def fd_second_derivative_weights(m_half):
    """Weights (c_0, c_1, ..., c_M) of the order-2M central second difference."""
    M = int(m_half)
    if M < 1:
        raise ValueError("order must be >= 2")
    c = [0.0] * (M + 1)
    for j in range(1, M + 1):
        c[j] = 2.0 * (-1) ** (j + 1) * factorial(M) ** 2 / (
            j * j * factorial(M - j) * factorial(M + j))
    c[0] = -2.0 * sum(c[1:])
    return np.array(c)


def second_difference(f, axis, h, m_half, periodic):
    """d^2 f / dx_axis^2 by the order-2M central difference with ghosts."""
    c = fd_second_derivative_weights(m_half)
    M = len(c) - 1
    pad = [(0, 0)] * f.ndim
    pad[axis] = (M, M)
    g = np.pad(f, pad, mode="wrap" if periodic else "edge")
    n = f.shape[axis]
    out = c[0] * f
    for j in range(1, M + 1):
        plus = np.take(g, np.arange(M + j, M + j + n), axis=axis)
        minus = np.take(g, np.arange(M - j, M - j + n), axis=axis)
        out = out + c[j] * (plus + minus)
    return out / (h * h)


def periodic_axes(bc):
    """Axes (of a (nz, ny, nx) array) that are periodic under bc."""
    if bc == BC_FREE:
        return ()
    if bc == BC_SURFACE:
        return (1, 2)
    if bc == BC_WIRE:
        return (0,)
    if bc == BC_PERIODIC:
        return (0, 1, 2)
    raise ValueError(bc)


def laplacian_fd(f, h, m_half, bc):
    per = periodic_axes(bc)
    return sum(second_difference(f, ax, h, m_half, ax in per) for ax in range(3))


def laplacian_spectral(f, h):
    """Periodic spectral Laplacian F^-1[-|k|^2 F f]."""
    nz, ny, nx = f.shape
    kz = wavenumbers(nz, h)[:, None, None]
    ky = wavenumbers(ny, h)[None, :, None]
    kx = rwavenumbers(nx, h)[None, None, :]
    k2 = kz * kz + ky * ky + kx * kx
    return sfft.irfftn(-k2 * sfft.rfftn(f), s=f.shape)


def q_field(eps, h, bc, fd_order=16):
    """q = sqrt(eps) * lap sqrt(eps)  (Eq. corr)."""
    if fd_order % 2:
        raise ValueError("fd_order must be even")
    s = np.sqrt(np.asarray(eps, dtype=np.float64))
    if bc == BC_PERIODIC:
        return s * laplacian_spectral(s, h)
    return s * laplacian_fd(s, h, fd_order // 2, bc)
