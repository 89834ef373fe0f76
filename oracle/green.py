"""Vacuum Poisson solver G_bc of the oracle (test infrastructure only).

G_bc maps a charge-like field f to the potential u that solves the standard
Poisson equation lap u = -4 pi f (Eq. SPe, Sec. II) under free, surface or
periodic boundary conditions.  In the paper this role is played by the ISF
Poisson solver (Sec. II.C); the ISF kernel itself is defined in a cited work,
not in the paper, so the discretisation used here is a cell-averaged Coulomb
kernel on a cell-centred grid:

  free      u_i = h^3 sum_j K(i - j) f_j ,  K(m) = I(m) / h ,
            I(m) = integral over the unit cube centred at m of 1/|u| d^3u ,
            evaluated through zero padding to (2nz, 2ny, 2nx) (Hockney).
  periodic  u = F^-1[ 4 pi / |k|^2  F f ],  zero at k = 0.
  wire      z spectral (periodic); in x, y, for each kz, the cell average of
            2 K0(|kz| rho) (kz != 0) or -2 ln(rho/Rw) (kz = 0), zero-padded to
            (2ny, 2nx) (oracle/wire.py).
  surface   x, y spectral (periodic); along z, for each in-plane wavevector
            k_par the cell average of the 1D Green's function
            g(k_par, z) = (2 pi / k_par) exp(-k_par |z|)     (k_par > 0),
            g(0, z)     = 2 pi (Lz - |z|),  Lz = 2 nz h          (k_par = 0),
            applied as a zero-padded (2 nz) convolution in z.

Surface k_par = 0 mode.  The 1D Green's function of d^2/dz^2 is -2 pi |z| up
to a constant.  Unshifted, the discrete operator has one negative eigenvalue
and PCG breaks down; shifted by 2 pi Lz it is non-negative on the whole padded
period (a tent) and the discrete G is positive definite.  A constant shift
adds C * (total charge of the k_par = 0 mode), which vanishes for the neutral
effective charge of a converged neutral problem, so the continuum solution is
unchanged.

Periodic k = 0 mode.  G drops it (value 0).  For linear Poisson-Boltzmann the
operator is non-singular and the preconditioner must be too: the k = 0
multiplier is then 4 pi / <kappa2/eps>, the screened-Poisson value for the
mean (apply(..., periodic_k0=...)).

All functions work in binary64.  Array shape convention: (nz, ny, nx).
"""
import numpy as np
from scipy import fft as sfft

from . import BC_FREE, BC_SURFACE, BC_PERIODIC, BC_WIRE

# Cells with max_a |m_a| <= NEAR_CUTOFF use the exact cube integral; the
# others use the multipole expansion of the cube average.  At the cutoff the
# two agree to ~3e-11 relative (tests/test_oracle_green.py).
NEAR_CUTOFF = 8


# --------------------------------------------------------------------------
# cell-averaged 1/r
# --------------------------------------------------------------------------
def _prism_antiderivative(x, y, z):
    """F(x, y, z) with d^3 F / dx dy dz = 1 / sqrt(x^2 + y^2 + z^2).

    Valid for x, y, z all nonzero (the callers only pass half-integers).
    """
    r = np.sqrt(x * x + y * y + z * z)
    return (y * z * np.log(x + r) + x * z * np.log(y + r) + x * y * np.log(z + r)
            - 0.5 * x * x * np.arctan(y * z / (x * r))
            - 0.5 * y * y * np.arctan(x * z / (y * r))
            - 0.5 * z * z * np.arctan(x * y / (z * r)))


def cube_integral_exact(mx, my, mz):
    """I(m): integral of 1/|u| over the unit cube centred at integer m.

    Inclusion-exclusion of the antiderivative over the 8 cube corners.  By
    symmetry I depends on |m_a| only, so the corners are at |m_a| +- 1/2.
    """
    mx = np.abs(np.asarray(mx, dtype=np.float64))
    my = np.abs(np.asarray(my, dtype=np.float64))
    mz = np.abs(np.asarray(mz, dtype=np.float64))
    total = np.zeros(np.broadcast(mx, my, mz).shape)
    for sx in (0, 1):
        for sy in (0, 1):
            for sz in (0, 1):
                sign = 1.0 if (sx + sy + sz) % 2 == 1 else -1.0
                total = total + sign * _prism_antiderivative(
                    mx - 0.5 + sx, my - 0.5 + sy, mz - 0.5 + sz)
    return total


def cube_integral_far(mx, my, mz):
    """Expansion of I(m) for |m| large: 1/r plus the r^-5 and r^-7 terms.

    The cube average of a function equals prod_a sinh(d_a/2)/(d_a/2) applied
    to it; for the harmonic 1/r the second-order term vanishes and the
    fourth- and sixth-order terms reduce to the polynomials below.
    """
    x = np.asarray(mx, dtype=np.float64)
    y = np.asarray(my, dtype=np.float64)
    z = np.asarray(mz, dtype=np.float64)
    x2, y2, z2 = x * x, y * y, z * z
    r2 = x2 + y2 + z2
    r = np.sqrt(r2)
    s4 = x2 * x2 + y2 * y2 + z2 * z2
    p22 = x2 * y2 + x2 * z2 + y2 * z2
    t4 = (-7.0 / 480.0 * s4 + 7.0 / 160.0 * p22) / (r2 ** 4 * r)
    s6 = x2 ** 3 + y2 ** 3 + z2 ** 3
    p42 = x2 * x2 * (y2 + z2) + y2 * y2 * (x2 + z2) + z2 * z2 * (x2 + y2)
    t6 = (2.0 * s6 - 15.0 * p42 + 180.0 * x2 * y2 * z2) / 1344.0 / (r2 ** 6 * r)
    return 1.0 / r + t4 + t6


def cell_averaged_inverse_distance(mx, my, mz):
    """I(m) by the rule: exact near the origin, expansion beyond NEAR_CUTOFF."""
    mx, my, mz = np.broadcast_arrays(np.abs(np.asarray(mx)), np.abs(np.asarray(my)),
                                     np.abs(np.asarray(mz)))
    near = np.maximum(np.maximum(mx, my), mz) <= NEAR_CUTOFF
    out = np.empty(mx.shape, dtype=np.float64)
    out[near] = cube_integral_exact(mx[near], my[near], mz[near])
    far = ~near
    out[far] = cube_integral_far(mx[far], my[far], mz[far])
    return out


def _padded_offsets(n):
    """|offset| of each index of a length-2n cyclic axis (index n maps to n)."""
    i = np.arange(2 * n)
    return np.where(i <= n, i, 2 * n - i)


def free_kernel_table(shape, h):
    """K(m) = I(m)/h on the (2nz, 2ny, 2nx) cyclic padded grid (even in m)."""
    nz, ny, nx = shape
    mz = _padded_offsets(nz)[:, None, None]
    my = _padded_offsets(ny)[None, :, None]
    mx = _padded_offsets(nx)[None, None, :]
    return cell_averaged_inverse_distance(mx, my, mz) / h


# --------------------------------------------------------------------------
# surface BC: 1D kernels along z
# --------------------------------------------------------------------------
def surface_z_kernel(kpar, m, h, k0_offset=0.0):
    """Cell average over z of the 1D Green's function, at integer offsets m.

    kpar > 0: average of (2 pi/k) exp(-k |z|) over [m h - h/2, m h + h/2];
    kpar = 0: average of -2 pi |z| (+ k0_offset) over the same cell.
    """
    kpar = np.asarray(kpar, dtype=np.float64)
    am = np.abs(np.asarray(m, dtype=np.float64))
    kpar, am = np.broadcast_arrays(kpar, am)
    out = np.empty(kpar.shape, dtype=np.float64)
    zero = kpar == 0.0
    # k_par = 0
    out[zero] = np.where(am[zero] == 0.0, -2.0 * np.pi * h / 4.0,
                         -2.0 * np.pi * h * am[zero]) + k0_offset
    k = kpar[~zero]
    a = am[~zero]
    centre = 4.0 * np.pi / (k * k * h) * (-np.expm1(-k * h / 2.0))
    off = (2.0 * np.pi / (k * k * h)) * np.exp(-k * (a * h - h / 2.0)) * (-np.expm1(-k * h))
    out[~zero] = np.where(a == 0.0, centre, off)
    return out


def surface_default_offset(nz, h):
    """2 pi Lz with Lz = 2 nz h, the padded z period."""
    return 2.0 * np.pi * (2 * nz * h)


def wavenumbers(n, h):
    """Angular wavenumbers 2 pi j / (n h) in numpy FFT order."""
    return 2.0 * np.pi * sfft.fftfreq(n, d=h)


def rwavenumbers(n, h):
    return 2.0 * np.pi * sfft.rfftfreq(n, d=h)


# --------------------------------------------------------------------------
# the solver object
# --------------------------------------------------------------------------
class VacuumSolver:
    """u = G_bc f on a (nz, ny, nx) cell-centred grid of spacing h."""

    def __init__(self, shape, h, bc, surface_k0_offset=None, workers=None):
        if bc not in (BC_FREE, BC_SURFACE, BC_PERIODIC, BC_WIRE):
            raise ValueError("unknown boundary condition %r" % (bc,))
        self.shape = tuple(int(s) for s in shape)
        self.h = float(h)
        self.bc = bc
        self.workers = workers
        nz, ny, nx = self.shape
        if bc == BC_FREE:
            self.fft_shape = (2 * nz, 2 * ny, 2 * nx)
            kern = free_kernel_table(self.shape, h)
            self.spectrum = h ** 3 * sfft.rfftn(kern, workers=workers).real
        elif bc == BC_WIRE:
            from . import wire
            self.fft_shape = (nz, 2 * ny, 2 * nx)
            self.spectrum = wire.wire_spectrum(self.shape, h)
        elif bc == BC_PERIODIC:
            self.fft_shape = (nz, ny, nx)
            kz = wavenumbers(nz, h)[:, None, None]
            ky = wavenumbers(ny, h)[None, :, None]
            kx = rwavenumbers(nx, h)[None, None, :]
            k2 = kz * kz + ky * ky + kx * kx
            with np.errstate(divide="ignore"):
                spec = np.where(k2 > 0.0, 4.0 * np.pi / np.where(k2 > 0, k2, 1.0), 0.0)
            self.spectrum = spec
        else:
            self.fft_shape = (2 * nz, ny, nx)
            ky = wavenumbers(ny, h)[:, None]
            kx = rwavenumbers(nx, h)[None, :]
            kpar = np.sqrt(ky * ky + kx * kx)                       # (ny, nx//2+1)
            m = _padded_offsets(nz)[:, None, None]                 # (2nz,1,1)
            if surface_k0_offset is None:
                surface_k0_offset = surface_default_offset(nz, h)
            self.surface_k0_offset = surface_k0_offset
            g = surface_z_kernel(kpar[None, :, :], m, h, surface_k0_offset)
            self.spectrum = h * sfft.fft(g, axis=0, workers=workers).real

    def apply(self, f, periodic_k0=None):
        f = np.asarray(f, dtype=np.float64)
        assert f.shape == self.shape
        nz, ny, nx = self.shape
        spec = self.spectrum
        if periodic_k0 is not None and self.bc == BC_PERIODIC:
            spec = spec.copy()
            spec[0, 0, 0] = periodic_k0
        fh = sfft.rfftn(f, s=self.fft_shape, workers=self.workers)
        u = sfft.irfftn(fh * spec, s=self.fft_shape, workers=self.workers)
        return u[:nz, :ny, :nx].copy()

    __call__ = apply


# --------------------------------------------------------------------------
# dense O(N^2) forms of the same operators (tiny grids only)
# --------------------------------------------------------------------------
def _index_grid(shape):
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def dense_green_free(shape, h):
    """G_ij = h^3 K(i - j) written out pairwise (no FFT)."""
    i, j, k = _index_grid(shape)
    di = i[:, None] - i[None, :]
    dj = j[:, None] - j[None, :]
    dk = k[:, None] - k[None, :]
    return h ** 2 * cell_averaged_inverse_distance(di, dj, dk)


def dense_green_periodic(shape, h):
    """G_ij = (1/N) sum_{k != 0} (4 pi/|k|^2) cos(k . (r_i - r_j)), every k."""
    nz, ny, nx = shape
    n = nx * ny * nz
    i, j, k = _index_grid(shape)
    x, y, z = i * h, j * h, k * h
    g = np.zeros((n, n))
    for kz in wavenumbers(nz, h):
        for ky in wavenumbers(ny, h):
            for kx in wavenumbers(nx, h):
                k2 = kx * kx + ky * ky + kz * kz
                if k2 == 0.0:
                    continue
                ph = kx * x + ky * y + kz * z
                g += (4.0 * np.pi / k2) * np.cos(ph[:, None] - ph[None, :])
    return g / n


def dense_laplacian_periodic(shape, h):
    """Spectral Laplacian as a matrix: (1/N) sum_k (-|k|^2) cos(k.(r_i - r_j))."""
    nz, ny, nx = shape
    n = nx * ny * nz
    i, j, k = _index_grid(shape)
    x, y, z = i * h, j * h, k * h
    lap = np.zeros((n, n))
    for kz in wavenumbers(nz, h):
        for ky in wavenumbers(ny, h):
            for kx in wavenumbers(nx, h):
                ph = kx * x + ky * y + kz * z
                lap -= (kx * kx + ky * ky + kz * kz) * np.cos(ph[:, None] - ph[None, :])
    return lap / n


def dense_green_surface(shape, h, k0_offset=None):
    """G_ij = (h/(nx ny)) sum_{kx,ky} cos(k_par . (r_i - r_j)_par) g(k_par, k_i - k_j)."""
    nz, ny, nx = shape
    if k0_offset is None:
        k0_offset = surface_default_offset(nz, h)
    i, j, k = _index_grid(shape)
    x, y = i * h, j * h
    dk = k[:, None] - k[None, :]
    g = np.zeros((len(i), len(i)))
    for ky in wavenumbers(ny, h):
        for kx in wavenumbers(nx, h):
            kpar = np.sqrt(kx * kx + ky * ky)
            ph = kx * x + ky * y
            g += np.cos(ph[:, None] - ph[None, :]) * surface_z_kernel(kpar, dk, h, k0_offset)
    return g * h / (nx * ny)


def dense_green(shape, h, bc, surface_k0_offset=None):
    if bc == BC_FREE:
        return dense_green_free(shape, h)
    if bc == BC_PERIODIC:
        return dense_green_periodic(shape, h)
    if bc == BC_SURFACE:
        return dense_green_surface(shape, h, surface_k0_offset)
    if bc == BC_WIRE:
        from .wire import dense_green_wire
        return dense_green_wire(shape, h)
    raise ValueError(bc)
