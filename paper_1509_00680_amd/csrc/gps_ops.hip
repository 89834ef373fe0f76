// Pointwise and stencil kernels of the PCG solver (Algorithm PCG with the
// operator identity of Eq. corr / Eq. corrPB) and the ionic update of
// Algorithm SCPBimproved, plus the plan-time spectrum tables.
//
// Reductions are deterministic: every work-group writes one FP64 partial per
// quantity, and the consuming kernel sums the partials in a fixed order in
// every work-group that needs the scalar (no atomics, no cross-group fences).
#include "gps_iter.h"
#include "gps_launch.h"

namespace gps {


// ---------------------------------------------------------------------------
// plan-time spectra
// ---------------------------------------------------------------------------
// t[kz][ky][kx] = scale * Re full[kz][ky][kx], kz <= Lz/2, ky <= Ly/2 (the
// spectrum of a real kernel that is even along every axis).
__global__ void k_compress_table(const cplx<double>* __restrict__ full, int Kx, int Ly, int Lz,
                                 double scale, double* __restrict__ t64, float* __restrict__ t32) {
  const int Lyh = Ly / 2 + 1, Lzh = Lz / 2 + 1;
  const long long n = (long long)Lzh * Lyh * Kx;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(i % Kx);
    const int ky = (int)((i / Kx) % Lyh);
    const int kz = (int)(i / ((long long)Kx * Lyh));
    const double v = full[((size_t)kz * Ly + ky) * Kx + kx].x * scale;
    t64[i] = v;
    t32[i] = (float)v;
  }
}

void launch_compress_table(const cplx<double>* full, int Kx, int Ly, int Lz, double scale,
                           double* t64, float* t32, hipStream_t s) {
  const long long n = (long long)(Lz / 2 + 1) * (Ly / 2 + 1) * Kx;
  const int grid = (int)std::min<long long>((n + kThreads - 1) / kThreads, 65535);
  GPS_LAUNCH(k_compress_table, dim3(grid), dim3(kThreads), 0, s, full, Kx, Ly, Lz, scale,
                     t64, t32);
}

// Surface boundaries: for each in-plane wavevector (kx, ky folded) the cell
// average over z of the 1D Green's function, on the cyclic padded axis:
//   k > 0 : (2 pi/k) exp(-k |z|)          k = 0 : 2 pi (Lz h - |z|)
// buf[m][c], c = ky * Kx + kx, m in [0, Lz).
__global__ void k_surface_gen(cplx<double>* __restrict__ buf, int Kx, int Lyh, int Lz, int nx,
                              int ny, double h, double k0_offset) {
  const long long nc = (long long)Kx * Lyh;
  const long long n = nc * Lz;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(i % nc);
    const int m = (int)(i / nc);
    const int kx = c % Kx, ky = c / Kx;
    const double gx = 2.0 * kPi * kx / (nx * h), gy = 2.0 * kPi * ky / (ny * h);
    const double k = sqrt(gx * gx + gy * gy);
    const int nz = Lz / 2;
    const int am = m <= nz ? m : Lz - m;
    double g;
    if (k == 0.0) {
      g = (am == 0 ? -2.0 * kPi * h / 4.0 : -2.0 * kPi * h * am) + k0_offset;
    } else if (am == 0) {
      g = 4.0 * kPi / (k * k * h) * (-expm1(-k * h / 2.0));
    } else {
      g = 2.0 * kPi / (k * k * h) * exp(-k * (am * h - h / 2.0)) * (-expm1(-k * h));
    }
    buf[i] = cmk(g, 0.0);
  }
}

void launch_surface_gen(cplx<double>* buf, int Kx, int Lyh, int Lz, int nx, int ny, double h,
                        double k0_offset, hipStream_t s) {
  const long long n = (long long)Kx * Lyh * Lz;
  const int grid = (int)std::min<long long>((n + kThreads - 1) / kThreads, 65535);
  GPS_LAUNCH(k_surface_gen, dim3(grid), dim3(kThreads), 0, s, buf, Kx, Lyh, Lz, nx, ny, h,
                     k0_offset);
}

// Wire boundaries (periodic z, isolated x and y): for each z mode kz the
// in-plane Green's function of (-lap_xy + kz^2) u = 4 pi f,
//   g(rho) = 2 K0(|kz| rho)  (kz != 0),   g(rho) = -2 ln(rho / Rw)  (kz = 0),
// averaged over the h x h cell of each offset of the (2ny, 2nx) padded plane.
// Off-origin cells: 10 x 10 Gauss-Legendre points.  The origin cell: polar
// coordinates on its eight triangles, (8/h^2) int_0^{pi/4} dt int_0^{R(t)}
// g(rho) rho drho with R(t) = h/(2 cos t); with I0 and the series of K0 the
// rho integral is exact term by term, the t integral takes the same 10
// Gauss-Legendre points.  out[iz][iy][ix] (real, Lz x Ly x Lx).

// K0(x), x > 0.  x <= 2: K0 = -(ln(x/2) + gamma) I0(x) + sum_j t^j H_j/(j!)^2,
// t = x^2/4, H_j the harmonic numbers.  x > 2: the integral
// K0(x) = e^{-x} int_0^inf exp(-x (cosh s - 1)) ds by the trapezoidal rule
// with step tau = min(0.2, 0.7/sqrt(x)) (the integrand is analytic in a
// strip, so the error falls like exp(-2 pi d / tau); these steps keep it below
// ~1e-16 relative), summed until x (cosh s - 1) > 40.
__device__ double wire_k0(double x) {
  constexpr double kGamma = 0.57721566490153286061;
  if (x <= 2.0) {
    const double t = 0.25 * x * x;
    double term = 1.0, i0 = 1.0, tail = 0.0, hj = 0.0;
    for (int j = 1; j < 30; ++j) {
      term *= t / ((double)j * j);
      hj += 1.0 / j;
      i0 += term;
      tail += term * hj;
      if (term < 1e-18) break;
    }
    return -(log(0.5 * x) + kGamma) * i0 + tail;
  }
  if (x > 740.0) return 0.0;
  const double tau = fmin(0.2, 0.7 / sqrt(x));
  double sum = 0.5;
  for (int j = 1; j < 400; ++j) {
    const double e = x * (cosh(j * tau) - 1.0);
    if (e > 40.0) break;
    sum += exp(-e);
  }
  return exp(-x) * tau * sum;
}

__device__ double wire_g(double rho, double k, double rw) {
  return k == 0.0 ? -2.0 * log(rho / rw) : 2.0 * wire_k0(k * rho);
}

__device__ double wire_origin(double k, double h, double rw, const GLRule& gl) {
  constexpr double kGamma = 0.57721566490153286061;
  double acc = 0.0;
  for (int a = 0; a < kGLPoints; ++a) {
    const double th = (gl.t[a] + 1.0) * (kPi / 8.0);
    const double R = h / (2.0 * cos(th));
    const double lR = log(R);
    double inner;
    if (k == 0.0) {
      inner = R * R * (log(rw) - lR + 0.5);
    } else {
      inner = 0.0;
      double coef = 1.0, hj = 0.0, Rp = R * R;
      const double base = -kGamma - log(0.5 * k);
      for (int j = 0; j < 24; ++j) {
        if (j > 0) {
          hj += 1.0 / j;
          coef *= 0.25 * k * k / ((double)j * j);
          Rp *= R * R;
        }
        const double p = 2.0 * j + 2.0;
        inner += 2.0 * coef * Rp / p * (hj + base - lR + 1.0 / p);
      }
    }
    acc += gl.w[a] * (kPi / 8.0) * inner;
  }
  return 8.0 / (h * h) * acc;
}

__global__ void k_wire_gen(double* __restrict__ out, int Lx, int Ly, int Lz, int nx, int ny,
                           double h, double rw, GLRule gl) {
  const long long n = (long long)Lx * Ly * Lz;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % Lx);
    const int iy = (int)((i / Lx) % Ly);
    const int iz = (int)(i / ((long long)Lx * Ly));
    const int mx = ix <= nx ? ix : Lx - ix;
    const int my = iy <= ny ? iy : Ly - iy;
    const int mz = iz <= Lz - iz ? iz : Lz - iz;
    const double k = 2.0 * kPi * mz / (Lz * h);
    double v;
    if (mx == 0 && my == 0) {
      v = wire_origin(k, h, rw, gl);
    } else {
      double acc = 0.0;
      for (int a = 0; a < kGLPoints; ++a) {
        const double x = (mx + 0.5 * gl.t[a]) * h;
        double row = 0.0;
        for (int b = 0; b < kGLPoints; ++b) {
          const double y = (my + 0.5 * gl.t[b]) * h;
          row += gl.w[b] * wire_g(sqrt(x * x + y * y), k, rw);
        }
        acc += gl.w[a] * row;
      }
      v = 0.25 * acc;
    }
    out[i] = v;
  }
}

void launch_wire_gen(double* out, const Geom& g, double rw, const GLRule& gl, hipStream_t s) {
  const long long n = (long long)g.Lx * g.Ly * g.Lz;
  const int grid = (int)std::min<long long>((n + kThreads - 1) / kThreads, 65535);
  GPS_LAUNCH(k_wire_gen, dim3(grid), dim3(kThreads), 0, s, out, g.Lx, g.Ly, g.Lz, g.nx, g.ny,
             g.h, rw, gl);
}

// t[kz][ky][kx] = scale * Re buf[kz][ky * Kx + kx], kz <= Lz/2
__global__ void k_surface_compress(const cplx<double>* __restrict__ buf, int Kx, int Lyh, int Lz,
                                   double scale, double* __restrict__ t64,
                                   float* __restrict__ t32) {
  const long long nc = (long long)Kx * Lyh;
  const long long n = nc * (Lz / 2 + 1);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = buf[i].x * scale;
    t64[i] = v;
    t32[i] = (float)v;
  }
}

void launch_surface_compress(const cplx<double>* buf, int Kx, int Lyh, int Lz, double scale,
                             double* t64, float* t32, hipStream_t s) {
  const long long n = (long long)Kx * Lyh * (Lz / 2 + 1);
  const int grid = (int)std::min<long long>((n + kThreads - 1) / kThreads, 65535);
  GPS_LAUNCH(k_surface_compress, dim3(grid), dim3(kThreads), 0, s, buf, Kx, Lyh, Lz, scale,
                     t64, t32);
}

// Periodic boundaries: 4 pi/|k|^2 (Green) or -|k|^2 (Laplacian), divided by
// the number of points (the inverse transform is unnormalised).  k = 0 -> 0.
__global__ void k_periodic_table(Geom g, int laplacian, double* __restrict__ t64,
                                 float* __restrict__ t32) {
  const int Lyh = g.Ly / 2 + 1, Lzh = g.Lz / 2 + 1;
  const long long n = (long long)Lzh * Lyh * g.Kx;
  const double norm = 1.0 / ((double)g.Lx * g.Ly * g.Lz);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(i % g.Kx);
    const int ky = (int)((i / g.Kx) % Lyh);
    const int kz = (int)(i / ((long long)g.Kx * Lyh));
    const double ax = 2.0 * kPi * kx / (g.Lx * g.h);
    const double ay = 2.0 * kPi * ky / (g.Ly * g.h);
    const double az = 2.0 * kPi * kz / (g.Lz * g.h);
    const double k2 = ax * ax + ay * ay + az * az;
    double v;
    if (laplacian) v = -k2 * norm;
    else v = k2 > 0.0 ? 4.0 * kPi / k2 * norm : 0.0;
    t64[i] = v;
    t32[i] = (float)v;
  }
}

void launch_periodic_table(const Geom& g, int laplacian, double* t64, float* t32, hipStream_t s) {
  const long long n = (long long)(g.Lz / 2 + 1) * (g.Ly / 2 + 1) * g.Kx;
  const int grid = (int)std::min<long long>((n + kThreads - 1) / kThreads, 65535);
  GPS_LAUNCH(k_periodic_table, dim3(grid), dim3(kThreads), 0, s, g, laplacian, t64, t32);
}

// ---------------------------------------------------------------------------
// solve-state reset (a kernel rather than a memset, so it may sit in a graph)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_reset_state(SlotTable<T> tab, Batch b, double abs_thr, double rel_thr,
                              int rel_from_b) {
  if (threadIdx.x == 0) {
    SolveState* st = tab.s[b.slot[blockIdx.x]].st;
    SolveState z{};
    z.abs_thr = abs_thr;
    z.rel_thr = rel_thr;
    z.rel_from_b = rel_from_b;
    *st = z;
  }
}

template <typename T>
void launch_reset_state(const SlotTable<T>& tab, const Batch& b, double abs_thr, double rel_thr,
                        int rel_from_b, hipStream_t s) {
  GPS_LAUNCH((k_reset_state<T>), dim3(b.n), dim3(64), 0, s, tab, b, abs_thr, rel_thr, rel_from_b);
}

// A free batch slot: its state says done, so every pass returns at once.
template <typename T>
__global__ void k_idle_state(SlotTable<T> tab, Batch b) {
  if (threadIdx.x == 0) {
    SolveState z{};
    z.done = 1;
    *tab.s[b.slot[blockIdx.x]].st = z;
  }
}

template <typename T>
void launch_idle_state(const SlotTable<T>& tab, const Batch& b, hipStream_t s) {
  GPS_LAUNCH((k_idle_state<T>), dim3(b.n), dim3(64), 0, s, tab, b);
}

// Periodic boundaries with ions: the k = 0 multiplier 4 pi / mean(kappa2/eps)
// (divided by the transform size) from the partials of the q kernel (one per
// q work-group).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_set_g0(SlotTable<T> tab, Batch b, int nparts,
                                                     double npts, double norm) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.x]];
  const double sum = sum_partials(sl.part_aux, nparts, 1);
  if (threadIdx.x == 0) {
    const double mean = sum / npts;
    sl.st->g0 = mean > 0.0 ? 4.0 * kPi / mean * norm : 0.0;
  }
}

template <typename T>
void launch_set_g0(const SlotTable<T>& tab, const Batch& b, long long n, double norm,
                   hipStream_t s) {
  GPS_LAUNCH((k_set_g0<T>), dim3(b.n), dim3(kThreads), 0, s, tab, b, qfield_groups(n),
                     double(n), norm);
}

// ---------------------------------------------------------------------------
// per-solve initialisation: sqrt(eps), 1/sqrt(eps), r0 = -4 pi rho, phi = 0
// partials (4 per group): ||r0||^2, sum rho, sum |rho|, sum rho^2
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_init(SlotTable<T> tab, Batch b,
                                                   const double* __restrict__ rho,
                                                   const double* __restrict__ eps, long long n,
                                                   int keep_src) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  // XCD-contiguous chunks: each XCD works on the same 1/8 of the grid as the
  // x passes, so fields written by one kernel are read from the same L2
  const long long base =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * kThreads * kVec + threadIdx.x;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int err = 0;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) {
      const double rv = rho[i], ev = eps[i];
      if (!(ev > 0.0)) err |= kErrEpsNonPositive;
      if (!isfinite(rv) || !isfinite(ev)) err |= kErrNonFinite;
      const double sq = sqrt(ev);
      sl.sq64[i] = sq;
      sl.isq[i] = T(1.0 / sq);
      if (sl.s) sl.s[i] = T(sq);
      const T r0 = T(-kFourPi * rv);
      sl.r[i] = r0;
      sl.phi[i] = 0.0;
      if (sl.src64 && !keep_src) sl.src64[i] = 0.0;   // (kept: warm start from s)
      a0 += double(r0) * double(r0);
      a1 += rv;
      a2 += fabs(rv);
      a3 += rv * rv;
    }
  }
  if (err) atomicOr(&sl.st->err, err);
  a0 = block_sum(a0);
  a1 = block_sum(a1);
  a2 = block_sum(a2);
  a3 = block_sum(a3);
  if (threadIdx.x == 0) {
    double* pp = sl.part_init + (size_t)blockIdx.x * 4;
    pp[0] = a0;
    pp[1] = a1;
    pp[2] = a2;
    pp[3] = a3;
  }
}

template <typename T>
void launch_init(const SlotTable<T>& tab, const Batch& b, const double* rho, const double* eps,
                 long long n, int keep_src, hipStream_t s) {
  GPS_LAUNCH((k_init<T>), dim3(vec_groups(n), b.n), dim3(kThreads), 0, s, tab, b, rho,
                     eps, n, keep_src);
}

// ---------------------------------------------------------------------------
// q + kappa2:  q = sqrt(eps) * lap_h sqrt(eps)  (Eq. corr), lap_h the order-2M
// central difference (edge-replicated ghosts on free axes, wrapped on
// periodic ones) or, when lap_sq is given, the spectral Laplacian computed by
// the FFT passes.  kappa2 = kappa_coef * gamma (Eq. corrPB).
// ---------------------------------------------------------------------------
struct FdWeights { double c[9]; };

// Stencil form (free and surface boundaries), 2.5D: a work-group owns a
// kQTX x kQTY column tile and marches along z over zlen planes.  The x and y
// neighbours of a plane come from an LDS tile with an M-wide halo (no
// corners), the z neighbours from a register queue of 2M+1 planes per
// thread, so a point costs about (2M + zlen)/zlen + 1.5 global loads instead
// of 6M + 1.  The next plane's halo and queue entry are loaded while the
// current plane is differenced.  zlen is chosen per grid (stencil_zlen): as
// long as the launch still has about two work-groups per CU, so the queue
// refill is amortized over long marches on large grids.
constexpr int kQTX = 32, kQTY = 16;
constexpr int kQThreads = kQTX * kQTY;

// Planes per z march of a 2.5D stencil over ntxy column tiles: the longest
// (up to 32, at least 4) that keeps about 512 work-groups.
int stencil_zlen(long long ntxy, int nz) {
  long long z = (ntxy * nz + 511) / 512;
  z = std::max<long long>(4, std::min<long long>(32, z));
  return (int)std::min<long long>(z, nz);
}

template <typename T, int M>
__global__ __launch_bounds__(kQThreads) void k_qstencil(SlotTable<T> tab, Batch b, Geom g,
                                                        FdWeights w, int ntx, int nty,
                                                        int zlen, double kappa_coef,
                                                        const double* __restrict__ eps,
                                                        const double* __restrict__ gamma,
                                                        double eps_bulk) {
  constexpr int TW = kQTX + 2 * M;                 // LDS tile width (x) and height (y)
  constexpr int TH = kQTY + 2 * M;
  constexpr int NXH = 2 * M * kQTY;                // halo slots left and right of the tile
  constexpr int NH = NXH + 2 * M * kQTX;           // ... plus above and below
  constexpr int HS = (NH + kQThreads - 1) / kQThreads;
  __shared__ double tile[TH * TW];
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  const double* __restrict__ sq = sl.sq64;
  const int tid = threadIdx.x;
  const int tx = tid % kQTX, ty = tid / kQTX;
  const int t = xcd_tile(blockIdx.x, gridDim.x);   // x fastest, then y, then z chunk
  const int ntxy = ntx * nty;
  const int zc = t / ntxy;
  const int yt = (t - zc * ntxy) / ntx;
  const int xt = t - zc * ntxy - yt * ntx;
  const int x0 = xt * kQTX, y0 = yt * kQTY, z0 = zc * zlen;
  const int z1 = min(z0 + zlen, g.nz);
  const int X = x0 + tx, Y = y0 + ty;
  const int plane = g.nx * g.ny;
  const int cxy = ghost_index(Y, g.ny, g.periodic_y) * g.nx + ghost_index(X, g.nx, g.periodic_x);
  // this thread's halo slots: LDS position and in-plane source offset
  int hl[HS], ho[HS];
#pragma unroll
  for (int s = 0; s < HS; ++s) {
    const int j = min(tid + s * kQThreads, NH - 1);   // surplus threads repeat the last slot
    int hx, hy;
    if (j < NXH) {
      const int row = j / (2 * M), c = j - (j / (2 * M)) * (2 * M);
      hx = c < M ? c : c + kQTX;
      hy = M + row;
    } else {
      const int jj = j - NXH;
      const int row = jj / kQTX, c = jj - (jj / kQTX) * kQTX;
      hx = M + c;
      hy = row < M ? row : row + kQTY;
    }
    hl[s] = hy * TW + hx;
    ho[s] = ghost_index(y0 - M + hy, g.ny, g.periodic_y) * g.nx +
            ghost_index(x0 - M + hx, g.nx, g.periodic_x);
  }
  // queue: qv[k] holds plane z - M + k of this thread's column
  double qv[2 * M + 1];
#pragma unroll
  for (int k = 0; k <= 2 * M; ++k)
    qv[k] = sq[(size_t)ghost_index(z0 - M + k, g.nz, g.periodic_z) * plane + cxy];
  double hv[HS];
#pragma unroll
  for (int s = 0; s < HS; ++s) hv[s] = sq[(size_t)z0 * plane + ho[s]];
  const double ih2 = 1.0 / (g.h * g.h);
  const bool out = X < g.nx && Y < g.ny;
  for (int z = z0; z < z1; ++z) {
    tile[(M + ty) * TW + M + tx] = qv[M];
#pragma unroll
    for (int s = 0; s < HS; ++s) tile[hl[s]] = hv[s];
    __syncthreads();
    // next plane's halo and queue entry, in flight while this plane is differenced
    const int zn = min(z + 1, g.nz - 1);
    double hn[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) hn[s] = sq[(size_t)zn * plane + ho[s]];
    const double qn = sq[(size_t)ghost_index(z + 1 + M, g.nz, g.periodic_z) * plane + cxy];
    double gv = 0.0;
    if (kappa_coef != 0.0 && out) {
      const size_t i = (size_t)z * plane + (size_t)Y * g.nx + X;
      gv = gamma ? gamma[i] : (eps[i] - 1.0) / (eps_bulk - 1.0);
    }
    const double* c = &tile[(M + ty) * TW + M + tx];
    // the rounding order is fixed: the centre product, then one fused
    // multiply-add per distance m over (x pair + y pair) + z pair
    double acc = __dmul_rn(3.0 * w.c[0], qv[M]);
#pragma unroll
    for (int m = 1; m <= M; ++m)
      acc = fma(w.c[m], ((c[m] + c[-m]) + (c[m * TW] + c[-m * TW])) + (qv[M + m] + qv[M - m]), acc);
    if (out) {
      const double lap = acc * ih2;
      double q = qv[M] * lap;
      if (kappa_coef != 0.0) q = __dadd_rn(q, __dmul_rn(kappa_coef, gv));
      const size_t o = (size_t)z * plane + (size_t)Y * g.nx + X;
      sl.qk[o] = T(q);
      if (sl.qk64) sl.qk64[o] = q;
    }
    __syncthreads();                              // tile reads done before the next writes
#pragma unroll
    for (int k = 0; k < 2 * M; ++k) qv[k] = qv[k + 1];
    qv[2 * M] = qn;
#pragma unroll
    for (int s = 0; s < HS; ++s) hv[s] = hn[s];
  }
}

// Spectral form (periodic): q = sqrt(eps) * lap_sq pointwise, one point per
// thread.  One kappa2/eps partial per work-group (the periodic k = 0
// multiplier).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_qfield(SlotTable<T> tab, Batch b, Geom g,
                                                     const double* __restrict__ lap_sq,
                                                     double kappa_coef,
                                                     const double* __restrict__ eps,
                                                     const double* __restrict__ gamma,
                                                     double eps_bulk) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  const int n = g.nx * g.ny * g.nz;
  const int i = xcd_tile(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  double kacc = 0.0;   // sum kappa2 / eps (periodic k = 0 multiplier)
  if (i < n) {
    double qv = sl.sq64[i] * lap_sq[i];
    if (kappa_coef != 0.0) {
      const double gm = gamma ? gamma[i] : (eps[i] - 1.0) / (eps_bulk - 1.0);
      const double k2 = kappa_coef * gm;
      qv += k2;
      kacc += k2 / eps[i];
    }
    sl.qk[i] = T(qv);
    if (sl.qk64) sl.qk64[i] = qv;
  }
  kacc = block_sum(kacc);
  if (threadIdx.x == 0) sl.part_aux[blockIdx.x] = kacc;
}

// Caller-supplied q (for instance the analytic q of a rigid cavity):
// q + kappa2 is q itself (no electrolyte on this path).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_qcopy(SlotTable<T> tab, Batch b, long long n,
                                                    const double* __restrict__ q) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  const long long base =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * kThreads * kVec + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) {
      const double v = q[i];
      sl.qk[i] = T(v);
      if (sl.qk64) sl.qk64[i] = v;
    }
  }
}

template <typename T>
void launch_qcopy(const SlotTable<T>& tab, const Batch& b, long long n, const double* q,
                  hipStream_t s) {
  GPS_LAUNCH((k_qcopy<T>), dim3(vec_groups(n), b.n), dim3(kThreads), 0, s, tab, b, n, q);
}

static FdWeights fd_weights(int M) {
  FdWeights w{};
  double fM = 1.0;
  for (int i = 2; i <= M; ++i) fM *= i;
  double sum = 0.0;
  for (int j = 1; j <= M; ++j) {
    double fa = 1.0, fb = 1.0;
    for (int i = 2; i <= M - j; ++i) fa *= i;
    for (int i = 2; i <= M + j; ++i) fb *= i;
    const double c = 2.0 * ((j + 1) % 2 == 0 ? 1.0 : -1.0) * fM * fM / (double(j) * j * fa * fb);
    w.c[j] = c;
    sum += c;
  }
  w.c[0] = -2.0 * sum;
  return w;
}

template <typename T>
void launch_qfield(const SlotTable<T>& tab, const Batch& b, const Geom& g, int fd_half,
                   const double* lap_sq, double kappa_coef, const double* eps,
                   const double* gamma, double eps_bulk, hipStream_t s) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  if (lap_sq) {
    GPS_LAUNCH((k_qfield<T>), dim3(qfield_groups(n), b.n), dim3(kThreads), 0, s, tab, b, g,
               lap_sq, kappa_coef, eps, gamma, eps_bulk);
    return;
  }
  const int ntx = (g.nx + kQTX - 1) / kQTX, nty = (g.ny + kQTY - 1) / kQTY;
  const int zlen = stencil_zlen((long long)ntx * nty, g.nz);
  const int nzc = (g.nz + zlen - 1) / zlen;
  const dim3 grid(ntx * nty * nzc, b.n);
  const FdWeights w = fd_weights(fd_half);
#define GPS_QF(MM)                                                                        \
  case MM:                                                                                \
    GPS_LAUNCH((k_qstencil<T, MM>), grid, dim3(kQThreads), 0, s, tab, b, g, w, ntx, nty,  \
               zlen, kappa_coef, eps, gamma, eps_bulk);                                   \
    break;
  switch (fd_half) {
    GPS_QF(1) GPS_QF(2) GPS_QF(3) GPS_QF(4) GPS_QF(5) GPS_QF(6) GPS_QF(7) GPS_QF(8)
    default: break;
  }
#undef GPS_QF
}

// ---------------------------------------------------------------------------
// ionic update of Algorithm SCPBimproved (Eqs. rhoions, ionsconcPB/MPB):
//   new = gamma sum_i Z_i c_i e^{x_i} / D,  x_i = -Z_i phi / kT,
//   D = 1 (Boltzmann) or 1 + sum_j a_j (e^{x_j} - 1) (steric), evaluated with
//   numerator and denominator scaled by e^{-xm}, xm = max(0, max_j x_j);
//   ion <- eta new + (1 - eta) ion;  r -= 4 pi (ion_new - ion_old), i.e. the
//   next right-hand side r' + rho^ions_k - rho^ions_{k-1} in residual form.
// partials (4 per group): ||r||^2, 0, 0, ||ion_new - ion_old||^2
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_ion_update(SlotTable<T> tab, Batch b, long long n,
                                                         IonParams ip) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  // XCD-contiguous chunks: each XCD works on the same 1/8 of the grid as the
  // x passes, so fields written by one kernel are read from the same L2
  const long long base =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * kThreads * kVec + threadIdx.x;
  double a0 = 0.0, a3 = 0.0;
  const T fpi = T(kFourPi);
#pragma unroll 1
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i >= n) break;
    const double phi = sl.phi[i];
    const double gm = ip.gamma ? ip.gamma[i] : (ip.eps[i] - 1.0) / (ip.eps_bulk - 1.0);
    double xs[4];
    double xm = 0.0;
    for (int sp = 0; sp < ip.nspecies; ++sp) {
      xs[sp] = -ip.Z[sp] * phi / ip.kT;
      xm = fmax(xm, xs[sp]);
    }
    double num = 0.0, fresh;
    if (ip.steric) {
      double den = 1.0;
      double asum = 0.0;
      den = 0.0;
      for (int sp = 0; sp < ip.nspecies; ++sp) {
        const double e = exp(xs[sp] - xm);
        num += ip.Z[sp] * ip.c[sp] * e;
        den += ip.a[sp] * e;
        asum += ip.a[sp];
      }
      den += exp(-xm) * (1.0 - asum);
      fresh = gm * num / den;
    } else {
      for (int sp = 0; sp < ip.nspecies; ++sp) num += ip.Z[sp] * ip.c[sp] * exp(xs[sp]);
      fresh = gm * num;
    }
    const T old = sl.ion[i];
    const T nw = T(ip.eta * fresh + (1.0 - ip.eta) * double(old));
    sl.ion[i] = nw;
    const T d = nw - old;
    const T rn = sl.r[i] - fpi * d;
    sl.r[i] = rn;
    a0 += double(rn) * double(rn);
    a3 += double(d) * double(d);
  }
  a0 = block_sum(a0);
  a3 = block_sum(a3);
  if (threadIdx.x == 0) {
    double* pp = sl.part_init + (size_t)blockIdx.x * 4;
    pp[0] = a0;
    pp[1] = 0.0;
    pp[2] = 0.0;
    pp[3] = a3;
  }
}

template <typename T>
void launch_ion_update(const SlotTable<T>& tab, const Batch& b, long long n, const IonParams& ip,
                       int, hipStream_t s) {
  GPS_LAUNCH((k_ion_update<T>), dim3(vec_groups(n), b.n), dim3(kThreads), 0, s, tab, b,
                     n, ip);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_outer_decide(SlotTable<T> tab, Batch b, int n_parts,
                                                           double rho_norm, double tol,
                                                           double abs_thr, double rel_thr_next,
                                                           int last) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.x]];
  const double d2 = sum_partials(sl.part_init + 3, n_parts, 4);
  if (threadIdx.x == 0) {
    SolveState* st = sl.st;
    const double dn = sqrt(d2);
    int status = -1;
    if (!isfinite(d2)) status = GPS_E_NONFINITE;
    else if (dn <= tol * rho_norm) status = GPS_OK;
    else if (last) status = GPS_E_NOT_CONVERGED;
    const double res = rho_norm > 0.0 ? dn / rho_norm : dn;
    if (status >= 0) {
      st->outer_done = 1;
      st->outer_status = status;
      st->outer_res = res;
    } else {
      SolveState z{};
      z.abs_thr = abs_thr;
      z.rel_thr = rel_thr_next;
      z.outer_res = res;
      *st = z;
    }
  }
}

template <typename T>
void launch_outer_decide(const SlotTable<T>& tab, const Batch& b, int n_parts, double rho_norm,
                         double tol, double abs_thr, double rel_thr_next, int last,
                         hipStream_t s) {
  GPS_LAUNCH((k_outer_decide<T>), dim3(b.n), dim3(kThreads), 0, s, tab, b, n_parts, rho_norm,
             tol, abs_thr, rel_thr_next, last);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero_ion(SlotTable<T> tab, Batch b,
                                                       long long n) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  // XCD-contiguous chunks: each XCD works on the same 1/8 of the grid as the
  // x passes, so fields written by one kernel are read from the same L2
  const long long base =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * kThreads * kVec + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) sl.ion[i] = T(0);
  }
}

template <typename T>
void launch_zero_ion(const SlotTable<T>& tab, const Batch& b, long long n, hipStream_t s) {
  GPS_LAUNCH((k_zero_ion<T>), dim3(vec_groups(n), b.n), dim3(kThreads), 0, s, tab, b, n);
}

// ---------------------------------------------------------------------------
// energy partials: sum rho phi (2 per group in part_aux: sum rho phi, 0)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_energy(SlotTable<T> tab, Batch b,
                                                     const double* __restrict__ rho, long long n) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  // XCD-contiguous chunks: each XCD works on the same 1/8 of the grid as the
  // x passes, so fields written by one kernel are read from the same L2
  const long long base =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * kThreads * kVec + threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) acc += rho[i] * sl.phi[i];
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    sl.part_aux[(size_t)blockIdx.x * 2] = acc;
    sl.part_aux[(size_t)blockIdx.x * 2 + 1] = 0.0;
  }
}

template <typename T>
void launch_energy(const SlotTable<T>& tab, const Batch& b, const double* rho, long long n,
                   hipStream_t s) {
  GPS_LAUNCH((k_energy<T>), dim3(vec_groups(n), b.n), dim3(kThreads), 0, s, tab, b, rho, n);
}

// ---------------------------------------------------------------------------
// true-residual refinement, in FP64 (free and surface boundaries).  The
// search directions are preconditioner images of sources, p = S^-1 G sigma,
// so the iterate is sqrt(eps) phi = G s with s accumulated by the x passes.
// Given u = G s:  phi = u / sqrt(eps) and, with A = S L_G S - diag(q + kappa2)
// and L_G G = -4 pi I,  r = b - A phi = -4 pi rho + 4 pi sqrt(eps) s + (q + kappa2) phi.
// The next iteration restarts PCG from this residual (no update, beta = 0).
// final: only phi (the iterate returned on exit).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_refine(SlotTable<T> tab, Batch b,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ u, long long n,
                                                     int final_step) {
  const Slot<T> sl = tab.s[b.slot[blockIdx.y]];
  const long long base =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * kThreads * kVec + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) {
      const double sq = sl.sq64[i];
      const double ph = u[i] / sq;
      sl.phi[i] = ph;
      if (!final_step)
        sl.r[i] = T(-kFourPi * rho[i] + kFourPi * sq * sl.src64[i] + sl.qk64[i] * ph);
    }
  }
  if (!final_step && blockIdx.x == 0 && threadIdx.x == 0) sl.st->restart = 1;
}

template <typename T>
void launch_refine(const SlotTable<T>& tab, const Batch& b, const double* rho, const double* u,
                   long long n, int final_step, hipStream_t s) {
  GPS_LAUNCH((k_refine<T>), dim3(vec_groups(n), b.n), dim3(kThreads), 0, s, tab, b, rho, u, n,
             final_step);
}

#define GPS_INST(T)                                                                              \
  template void launch_reset_state<T>(const SlotTable<T>&, const Batch&, double, double, int,       \
                                      hipStream_t);                                              \
  template void launch_idle_state<T>(const SlotTable<T>&, const Batch&, hipStream_t);             \
  template void launch_set_g0<T>(const SlotTable<T>&, const Batch&, long long, double,            \
                                 hipStream_t);                                                   \
  template void launch_init<T>(const SlotTable<T>&, const Batch&, const double*, const double*,       \
                               long long, int, hipStream_t);                                          \
  template void launch_qfield<T>(const SlotTable<T>&, const Batch&, const Geom&, int, const double*,  \
                                 double, const double*, const double*, double, hipStream_t);     \
  template void launch_qcopy<T>(const SlotTable<T>&, const Batch&, long long, const double*,        \
                                hipStream_t);                                                    \
  template void launch_ion_update<T>(const SlotTable<T>&, const Batch&, long long, const IonParams&,  \
                                     int, hipStream_t);                                          \
  template void launch_zero_ion<T>(const SlotTable<T>&, const Batch&, long long, hipStream_t);        \
  template void launch_outer_decide<T>(const SlotTable<T>&, const Batch&, int, double, double, double, \
                                       double, int, hipStream_t);                                \
  template void launch_energy<T>(const SlotTable<T>&, const Batch&, const double*, long long,         \
                                 hipStream_t);                                                   \
  template void launch_refine<T>(const SlotTable<T>&, const Batch&, const double*, const double*,    \
                                 long long, int, hipStream_t);
GPS_INST(float)
GPS_INST(double)
#undef GPS_INST

}  // namespace gps
