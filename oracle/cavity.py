"""Rigid cavity and polarization charge in plain binary64 (test infrastructure only).

Rigid cavity, Sec. IV.A, Eq. RigCav: for atoms at R_i with cavity radii d_i
and one transition width Delta,
    eps(r) = (eps0 - 1) * prod_i h(d_i, Delta; |r - R_i|) + 1,
with the switch of Eq. hfunc, h(d, Delta; r) = (1 + erf((r - d)/Delta)) / 2.
The paper notes that every field depending on eps follows analytically; the
one the PCG needs is the correction vector of Eq. corr,
    q = sqrt(eps) lap sqrt(eps) = lap(eps)/2 - |grad eps|^2 / (4 eps),
written here with the product rule over the atoms (no logarithmic
derivatives, no divisions by h):
    H = prod_i h_i,   grad H = sum_i P_i grad h_i,
    lap H = sum_i P_i lap h_i + sum_{i != j} P_ij grad h_i . grad h_j,
where P_i (P_ij) is the product of the h_k with k != i (k != i, j), and for
one atom, with t = (r - d)/Delta,
    h'  = exp(-t^2) / (Delta sqrt(pi)),   h'' = -2 t h' / Delta,
    grad h = h' (r - R)/r,                lap h = h'' + 2 h'/r.
Reading: at a grid point that coincides with an atom centre (r = 0) the
radial switch has a cusp (h'(0) != 0); its gradient is taken as 0 and its
Laplacian as h''(0), i.e. the 2 h'/r term is dropped.  Distances along
periodic axes are minimum-image distances in the cell of n h.

Polarization charge, Sec. II.A: Eq. remap splits lap phi = -4 pi (rho/eps +
rho_iter) with rho_iter = (1/4 pi) grad ln eps . grad phi (Eq. rhoiter), and
equals -4 pi (rho + rho_pol).  Hence
    rho_pol = rho_iter - (1 - 1/eps) rho.
Eq. rhopol prints a plus sign before the second term; the sign above is the
one Eq. remap implies, and the physical one (the solvent screens the solute's
charge).  The gradients are order-2M central differences,
    f'(x) ~ (1/h) sum_{j=1..M} c_j (f(x + j h) - f(x - j h)),
    c_j = (-1)^(j+1) (M!)^2 / (j (M - j)! (M + j)!),
which are exact on polynomials of degree <= 2M, with the ghosts of the q
stencil: edge-replicated along free axes, wrapped along periodic ones.
"""
from math import factorial

import numpy as np
from scipy.special import erf

from .stencil import periodic_axes

SQRT_PI = np.sqrt(np.pi)


def _axis(n, h):
    return (np.arange(n) - (n - 1) / 2.0) * h


def rigid_cavity_points(x, y, z, atoms, delta, eps0, periodic=(False, False, False),
                        cell=(None, None, None)):
    """eps and q at the points (x, y, z) (arrays of one shape).

    atoms: (natoms, 4) array of (X, Y, Z, d).  periodic / cell: per axis
    (x, y, z), whether distances wrap and the cell length n h.
    """
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 4)
    na = len(atoms)
    hv, g, lap = [], [], []
    for X, Y, Z, d in atoms:
        comps = []
        for c, C, per, L in ((x, X, periodic[0], cell[0]), (y, Y, periodic[1], cell[1]),
                             (z, Z, periodic[2], cell[2])):
            dc = c - C
            if per:
                dc = dc - L * np.round(dc / L)
            comps.append(dc)
        r = np.sqrt(comps[0] ** 2 + comps[1] ** 2 + comps[2] ** 2)
        t = (r - d) / delta
        h0 = 0.5 * (1.0 + erf(t))
        h1 = np.exp(-t * t) / (delta * SQRT_PI)
        h2 = -2.0 * t / delta * h1
        pos = r > 0.0
        rs = np.where(pos, r, 1.0)
        g.append([np.where(pos, h1 * c / rs, 0.0) for c in comps])
        lap.append(h2 + np.where(pos, 2.0 * h1 / rs, 0.0))
        hv.append(h0)

    def prod_except(skip):
        out = np.ones_like(x)
        for k in range(na):
            if k not in skip:
                out = out * hv[k]
        return out

    H = prod_except(())
    gH = [np.zeros_like(x) for _ in range(3)]
    lH = np.zeros_like(x)
    for i in range(na):
        Pi = prod_except((i,))
        for a in range(3):
            gH[a] = gH[a] + Pi * g[i][a]
        lH = lH + Pi * lap[i]
        for j in range(na):
            if j != i:
                lH = lH + prod_except((i, j)) * (g[i][0] * g[j][0] + g[i][1] * g[j][1] +
                                                 g[i][2] * g[j][2])
    a = eps0 - 1.0
    eps = a * H + 1.0
    grad2 = a * a * (gH[0] ** 2 + gH[1] ** 2 + gH[2] ** 2)
    q = 0.5 * a * lH - grad2 / (4.0 * eps)
    return eps, q


def rigid_cavity(shape, h, atoms, delta, eps0, bc="free"):
    """Eq. RigCav on the cell-centred (nz, ny, nx) grid: returns (eps, q)."""
    nz, ny, nx = shape
    per_axes = periodic_axes(bc)              # numpy axes: 0 = z, 1 = y, 2 = x
    periodic = (2 in per_axes, 1 in per_axes, 0 in per_axes)
    cell = (nx * h, ny * h, nz * h)
    x = _axis(nx, h)[None, None, :] + np.zeros(shape)
    y = _axis(ny, h)[None, :, None] + np.zeros(shape)
    z = _axis(nz, h)[:, None, None] + np.zeros(shape)
    return rigid_cavity_points(x, y, z, atoms, delta, eps0, periodic, cell)


def fd_first_derivative_weights(m_half):
    """(c_1, ..., c_M) of the order-2M central first difference."""
    M = int(m_half)
    if M < 1:
        raise ValueError("order must be >= 2")
    return np.array([(-1) ** (j + 1) * factorial(M) ** 2 /
                     (j * factorial(M - j) * factorial(M + j)) for j in range(1, M + 1)],
                    dtype=np.float64)


def first_difference(f, axis, h, m_half, periodic):
    """df/dx_axis by the order-2M central difference with ghosts."""
    c = fd_first_derivative_weights(m_half)
    M = len(c)
    pad = [(0, 0)] * f.ndim
    pad[axis] = (M, M)
    g = np.pad(f, pad, mode="wrap" if periodic else "edge")
    n = f.shape[axis]
    out = np.zeros(f.shape)
    for j in range(1, M + 1):
        plus = np.take(g, np.arange(M + j, M + j + n), axis=axis)
        minus = np.take(g, np.arange(M - j, M - j + n), axis=axis)
        out = out + c[j - 1] * (plus - minus)
    return out / h


def gradient_fd(f, h, m_half, bc):
    per = periodic_axes(bc)
    return [first_difference(f, ax, h, m_half, ax in per) for ax in range(3)]


def polarization_charge(rho, eps, phi, h, bc, fd_order=16):
    """rho_pol = (1/4 pi) grad ln eps . grad phi - (1 - 1/eps) rho (Eqs. rhoiter,
    remap; the sign of Eq. rhopol as Eq. remap implies it)."""
    if fd_order % 2:
        raise ValueError("fd_order must be even")
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    ge = gradient_fd(np.log(eps), h, fd_order // 2, bc)
    gp = gradient_fd(phi, h, fd_order // 2, bc)
    rho_iter = (ge[0] * gp[0] + ge[1] * gp[1] + ge[2] * gp[2]) / (4.0 * np.pi)
    return rho_iter - (1.0 - 1.0 / eps) * rho
