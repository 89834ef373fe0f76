"""Wire boundary conditions for the vacuum solver (test infrastructure only).

Sec. II.C lists free, wire, surface and periodic boundary conditions for the
SPe solver.  Wire: periodic along z (period Lz = nz h), isolated along x and
y.  Along z the potential is expanded in the nz periodic modes kz; for each
mode the in-plane Green's function of (-lap_xy + kz^2) u = 4 pi f is
    g_kz(rho) = 2 K0(|kz| rho)       (kz != 0),
    g_0(rho)  = -2 ln(rho / Rw)      (kz = 0),
i.e. the z-Fourier transform of 1/|r| (the kz = 0 one up to a constant).
Rw = 2 h sqrt(nx^2 + ny^2), twice the largest in-plane distance on the padded
grid, so that g_0 > 0 there.  Like the surface BC's k_par = 0 shift, the
constant adds C * (charge per unit length of the kz = 0 mode) to the
potential, zero for a neutral effective charge.

Discretisation: u_i = (h^2 / nz) sum_j sum_kz cos(kz (z_i - z_j)) A_kz(i - j),
with A_kz(m) the average of g_kz over the h x h square centred on the
in-plane offset (mx h, my h), applied as a zero-padded (2ny, 2nx) convolution
in x and y and a periodic one in z.  Cell averages:
  * off-origin cells: 10-point Gauss-Legendre in x times 10-point in y;
  * the origin cell: polar coordinates on its eight triangles,
      A = (8/h^2) int_0^{pi/4} int_0^{R(t)} g(rho) rho drho dt,  R(t) = h / (2 cos t),
    where the rho integral is exact: with the series
      K0(x) = -(ln(x/2) + gamma) I0(x) + sum_{j>=1} (x/2)^(2j) H_j / (j!)^2
    (H_j the harmonic numbers), 2 K0(k rho) = sum_j (k/2)^(2j)/(j!)^2 rho^(2j)
    * 2 (H_j - gamma - ln(k/2) - ln rho), and
      int_0^R rho^(2j+1) (c - ln rho) drho = R^(2j+2)/(2j+2) (c - ln R + 1/(2j+2));
    the t integral is 10-point Gauss-Legendre.
"""
import numpy as np
from scipy.special import k0

EULER_GAMMA = 0.57721566490153286061
GL_POINTS = 10
SERIES_TERMS = 24


def wire_radius(nx, ny, h):
    """Rw of the kz = 0 kernel: twice the largest in-plane padded distance."""
    return 2.0 * h * np.sqrt(float(nx) ** 2 + float(ny) ** 2)


def _g(rho, kz, rw):
    """In-plane Green's function of mode kz at distances rho > 0."""
    if kz == 0.0:
        return -2.0 * np.log(rho / rw)
    return 2.0 * k0(abs(kz) * rho)


def _origin_average(kz, h, rw):
    t, w = np.polynomial.legendre.leggauss(GL_POINTS)
    theta = (t + 1.0) * (np.pi / 8.0)            # [0, pi/4]
    wt = w * (np.pi / 8.0)
    R = h / (2.0 * np.cos(theta))
    if kz == 0.0:
        inner = R * R * (np.log(rw) - np.log(R) + 0.5)
    else:
        k = abs(kz)
        inner = np.zeros_like(R)
        harmonic = 0.0
        coef = 1.0                                # (k/2)^(2j) / (j!)^2
        for j in range(SERIES_TERMS):
            if j > 0:
                harmonic += 1.0 / j
                coef *= (k / 2.0) ** 2 / (j * j)
            c = harmonic - EULER_GAMMA - np.log(k / 2.0)
            p = 2 * j + 2
            inner = inner + 2.0 * coef * R ** p / p * (c - np.log(R) + 1.0 / p)
    return 8.0 / (h * h) * np.sum(wt * inner)


def cell_average(mx, my, kz, h, rw):
    """A_kz(m): average of g_kz over the h x h cell centred on (mx h, my h)."""
    mx = np.asarray(mx, dtype=np.float64)
    my = np.asarray(my, dtype=np.float64)
    mx, my = np.broadcast_arrays(mx, my)
    t, w = np.polynomial.legendre.leggauss(GL_POINTS)
    out = np.empty(mx.shape)
    origin = (mx == 0.0) & (my == 0.0)
    xs = (mx[..., None] + 0.5 * t) * h            # (..., GL)
    ys = (my[..., None] + 0.5 * t) * h
    rho = np.sqrt(xs[..., :, None] ** 2 + ys[..., None, :] ** 2)
    rho = np.where(origin[..., None, None], 1.0, rho)     # origin cell handled below
    vals = _g(rho, kz, rw)
    out[...] = 0.25 * np.einsum("...ab,a,b->...", vals, w, w)
    if np.any(origin):
        out[origin] = _origin_average(kz, h, rw)
    return out


def _padded_offsets(n):
    i = np.arange(2 * n)
    return np.where(i <= n, i, 2 * n - i)


def wavenumbers(n, h):
    return 2.0 * np.pi * np.fft.fftfreq(n, d=h)


def wire_kernel_table(shape, h):
    """A_kz(m) for every kz (numpy FFT order) on the (2ny, 2nx) padded plane."""
    nz, ny, nx = shape
    rw = wire_radius(nx, ny, h)
    mx = _padded_offsets(nx)[None, :]
    my = _padded_offsets(ny)[:, None]
    return np.stack([cell_average(mx, my, kz, h, rw) for kz in wavenumbers(nz, h)])


def wire_spectrum(shape, h):
    """h^2 FFT_xy of the kernel table (real, even), shape (nz, 2ny, nx + 1)."""
    return h * h * np.fft.rfft2(wire_kernel_table(shape, h), axes=(1, 2)).real


def dense_green_wire(shape, h):
    """G_ij = (h^2/nz) sum_kz cos(kz (z_i - z_j)) A_kz(x_i - x_j, y_i - y_j)."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    rw = wire_radius(nx, ny, h)
    dx = np.abs(i[:, None] - i[None, :])
    dy = np.abs(j[:, None] - j[None, :])
    dz = (k[:, None] - k[None, :]) * h
    g = np.zeros((len(i), len(i)))
    mx = np.arange(nx)[None, :]
    my = np.arange(ny)[:, None]
    for kz in wavenumbers(nz, h):
        a = cell_average(mx, my, kz, h, rw)          # every in-plane offset once
        g += np.cos(kz * dz) * a[dy, dx]
    return g * h * h / nz
