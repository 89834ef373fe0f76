// Cavity builder, diagnostics and the comparison iterations around the PCG solve:
//  * the rigid cavity of Eq. RigCav (Sec. IV.A) with its analytic correction
//    vector q = sqrt(eps) lap sqrt(eps) (Eq. corr);
//  * the polarization charge of Eqs. rhoiter and remap,
//    rho_pol = (1/4 pi) grad ln eps . grad phi - (1 - 1/eps) rho,
//    with order-2M central first differences (the sign of the second term is
//    the one Eq. remap implies; Eq. rhopol prints a plus);
//  * the operator and pointwise steps of Algorithm SC and the PSD minimization
//    (Sec. II.A, Eq. PrePSD).
#include <mutex>

#include "gps.h"
#include "gps_device.h"
#include "gps_launch.h"

namespace gps {

// ---------------------------------------------------------------------------
// Rigid cavity.  With a = eps0 - 1, h_i = erfc(-t_i)/2, t_i = (r_i - d_i)/Delta
// (Eq. hfunc) and H = prod_i h_i:  eps = a H + 1 and
//   q = (a/2) lap H - a^2 |grad H|^2 / (4 eps).
// The derivatives of H go through the logarithmic derivatives
//   u_i = h_i'/h_i = 2 / (Delta sqrt(pi) erfcx(-t_i)),
// which stay finite where h_i underflows (deep inside an atom):
//   grad H = H G,  G = sum_i u_i (r - R_i)/r_i,
//   lap H  = H (|G|^2 + sum_i [u_i (2/r_i - 2 t_i/Delta) - u_i^2]).
// At r_i = 0 (a grid point on an atom centre) the radial switch has a cusp;
// its gradient is taken as 0 and its Laplacian as h_i''(0): the atom adds
// -2 t_i u_i/Delta only.  Periodic axes use minimum-image separations.
// An atom with t_i > kFarT contributes nothing: there erfc(-t_i)/2 rounds to
// 1 in binary64 and u_i Delta < 3e-19, so its terms in G and in the sum are
// below 1e-17 / Delta^2, far below the rounding of max|q| ~ (eps0 - 1)/Delta^2.  A work-group covers an 8 x 8 x 4 block of grid
// points (a wavefront an 8 x 8 patch of one plane), so the lanes of a
// wavefront are near the same atoms and skip the same ones.
constexpr double kFarT = 6.5;
constexpr int kCBX = 8, kCBY = 8, kCBZ = kThreads / (kCBX * kCBY);

__global__ __launch_bounds__(kThreads) void k_rigid_cavity(Geom g, int nbx, int nby,
                                                           const double* __restrict__ atoms,
                                                           int natoms, double delta, double eps0,
                                                           double* __restrict__ eps,
                                                           double* __restrict__ q) {
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int bz = b / (nbx * nby);
  const int by = (b - bz * nbx * nby) / nbx;
  const int bx = b - bz * nbx * nby - by * nbx;
  const int ix = bx * kCBX + tid % kCBX;
  const int iy = by * kCBY + (tid / kCBX) % kCBY;
  const int iz = bz * kCBZ + tid / (kCBX * kCBY);
  if (ix >= g.nx || iy >= g.ny || iz >= g.nz) return;
  const double x = (ix - 0.5 * (g.nx - 1)) * g.h;
  const double y = (iy - 0.5 * (g.ny - 1)) * g.h;
  const double z = (iz - 0.5 * (g.nz - 1)) * g.h;
  const double lx = g.nx * g.h, ly = g.ny * g.h, lz = g.nz * g.h;
  const double idelta = 1.0 / delta;
  const double cu = 2.0 / (delta * 1.7724538509055160273);   // 2 / (Delta sqrt(pi))
  double H = 1.0, gx = 0.0, gy = 0.0, gz = 0.0, w = 0.0;
  for (int a = 0; a < natoms; ++a) {
    const double* at = atoms + 4 * a;
    double dx = x - at[0], dy = y - at[1], dz = z - at[2];
    if (g.periodic_x) dx -= lx * rint(dx / lx);
    if (g.periodic_y) dy -= ly * rint(dy / ly);
    if (g.periodic_z) dz -= lz * rint(dz / lz);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double t = (r - at[3]) * idelta;
    if (t > kFarT) continue;
    H *= 0.5 * erfc(-t);
    const double u = cu / erfcx(-t);
    w -= 2.0 * t * u * idelta;
    if (r > 0.0) {
      const double ur = u / r;
      gx += ur * dx;
      gy += ur * dy;
      gz += ur * dz;
      w += 2.0 * ur - u * u;
    }
  }
  const size_t i = ((size_t)iz * g.ny + iy) * g.nx + ix;
  const double a = eps0 - 1.0;
  const double aH = a * H;
  const double e = aH + 1.0;
  eps[i] = e;
  if (q) {
    const double g2 = gx * gx + gy * gy + gz * gz;
    q[i] = 0.5 * aH * (g2 + w) - aH * aH * g2 / (4.0 * e);
  }
}

void launch_rigid_cavity(const Geom& g, const double* atoms, int natoms, double delta,
                         double eps0, double* eps, double* q, hipStream_t s) {
  const int nbx = (g.nx + kCBX - 1) / kCBX, nby = (g.ny + kCBY - 1) / kCBY;
  const int nbz = (g.nz + kCBZ - 1) / kCBZ;
  GPS_LAUNCH(k_rigid_cavity, dim3((unsigned)(nbx * nby * nbz)), dim3(kThreads), 0, s, g, nbx,
             nby, atoms, natoms, delta, eps0, eps, q);
}

// ---------------------------------------------------------------------------
// Stop decision of an SC/PSD step (one work-group): from the update's partial
// pairs (||r||^2, ||r/eps||^2) it records the step, its norms and the status,
// and sets done on convergence, failure or the step limit.  It acts only when
// the update has marked a decision pending, so every update is decided once,
// whether by the next step's operator launch or by a launch of its own.
// ---------------------------------------------------------------------------
__device__ void sc_decide_group(const double* __restrict__ part, int nparts, ScState* st) {
  if (st->done || !st->pending) return;          // the same for every thread
  const double rr = sum_partials(part, nparts, 2);
  const double ff = sum_partials(part + 1, nparts, 2);
  if (threadIdx.x != 0) return;
  ScState z = *st;
  z.pending = 0;
  if (z.status != GPS_E_NOT_CONVERGED) {          // breakdown or non-finite step
    z.done = 1;
    *st = z;
    return;
  }
  const int step = z.step;
  z.ff_prev = z.ff;
  z.rr = rr;
  z.ff = ff;
  z.step = step + 1;
  if (!isfinite(rr) || !isfinite(ff)) {
    z.status = GPS_E_NONFINITE;
  } else if (z.method == GPS_METHOD_SC) {
    // SC's residual ||rho_iter_{k+1} - rho_iter_k|| = (eta/4 pi) ||r_k/eps|| of
    // the iterate before this step; the first step is the unmixed phi_0
    if (step >= 1) {
      z.iters = step;
      if (z.eta / kFourPi * sqrt(z.ff_prev) <= z.thr_sc) z.status = GPS_OK;
    }
  } else {
    z.iters = step + 1;
    if (z.method == GPS_METHOD_PSD ? sqrt(rr) <= z.thr_r : sqrt(ff) <= z.thr_w) z.status = GPS_OK;
  }
  if (z.status != GPS_E_NOT_CONVERGED || z.step >= z.max_steps) z.done = 1;
  *st = z;
}

// ---------------------------------------------------------------------------
// Polarization charge.  First differences of order 2M:
//   f'(x) ~ (1/h) sum_{m=1..M} c_m (f(x + m h) - f(x - m h)),
//   c_m = (-1)^(m+1) (M!)^2 / (m (M - m)! (M + m)!),
// with the ghosts of the q stencil (edge-replicated on free axes, wrapped on
// periodic ones).  2.5D like the q stencil: a kPTX x kPTY column tile marches
// along z over zlen planes (stencil_zlen); x and y neighbours of ln eps and phi come from
// two LDS tiles with an M-wide halo, z neighbours from two register queues of
// 2M+1 planes, and the next plane's loads are in flight while the current
// one is differenced.  ln eps comes precomputed (k_log_field), and eps itself
// is read only at the tile's own points.
// ---------------------------------------------------------------------------
struct FdFirst { double c[9]; };

constexpr int kPTX = 32, kPTY = 8;
constexpr int kPThreads = kPTX * kPTY;

// AV = false: out = rho_pol from (rho, eps, phi).  AV = true (PSD / SC
// operator, Eq. PrePSD with grad eps = eps grad ln eps): with rho -> r and
// phi -> v, out = A v = -4 pi r + eps grad ln eps . grad v, and two FP64
// partials per work-group into part[2 b], part[2 b + 1]: (v, r) and (v, A v)
// (paper != 0: Algorithm PCG's step with beta = 0), else (A v, r/eps^2) and
// (A v, A v/eps^2) (the step that minimizes ||r/eps||_2).
template <int M, bool AV>
__global__ __launch_bounds__(kPThreads) void k_polarization(Geom g, FdFirst w, int ntx, int nty,
                                                            int zlen, int paper, const int* stop,
                                                            const double* __restrict__ rho,
                                                            const double* __restrict__ eps,
                                                            const double* __restrict__ lne,
                                                            const double* __restrict__ phi,
                                                            double* __restrict__ out,
                                                            double* __restrict__ part,
                                                            ScDecide dec) {
  constexpr int TW = kPTX + 2 * M;
  constexpr int TH = kPTY + 2 * M;
  constexpr int NXH = 2 * M * kPTY;                // halo slots left and right of the tile
  constexpr int NH = NXH + 2 * M * kPTX;           // ... plus above and below
  constexpr int HS = (NH + kPThreads - 1) / kPThreads;
  __shared__ double te[TH * TW];
  __shared__ double tp[TH * TW];
  // SC/PSD: work-group 0 takes the previous update's stop decision, the
  // tiles start at work-group 1
  const int d0 = dec.st ? 1 : 0;
  if (d0 && blockIdx.x == 0) {
    sc_decide_group(dec.part, dec.nparts, dec.st);
    return;
  }
  if (stop && *stop) return;
  const int tid = threadIdx.x;
  const int tx = tid % kPTX, ty = tid / kPTX;
  const int t = xcd_tile(blockIdx.x - d0, gridDim.x - d0);   // x fastest, then y, then z chunk
  const int ntxy = ntx * nty;
  const int zc = t / ntxy;
  const int yt = (t - zc * ntxy) / ntx;
  const int xt = t - zc * ntxy - yt * ntx;
  const int x0 = xt * kPTX, y0 = yt * kPTY, z0 = zc * zlen;
  const int z1 = min(z0 + zlen, g.nz);
  const int X = x0 + tx, Y = y0 + ty;
  const int plane = g.nx * g.ny;
  const int cxy = ghost_index(Y, g.ny, g.periodic_y) * g.nx + ghost_index(X, g.nx, g.periodic_x);
  int hl[HS], ho[HS];
#pragma unroll
  for (int s = 0; s < HS; ++s) {
    const int j = min(tid + s * kPThreads, NH - 1);   // surplus threads repeat the last slot
    int hx, hy;
    if (j < NXH) {
      const int row = j / (2 * M), c = j - (j / (2 * M)) * (2 * M);
      hx = c < M ? c : c + kPTX;
      hy = M + row;
    } else {
      const int jj = j - NXH;
      const int row = jj / kPTX, c = jj - (jj / kPTX) * kPTX;
      hx = M + c;
      hy = row < M ? row : row + kPTY;
    }
    hl[s] = hy * TW + hx;
    ho[s] = ghost_index(y0 - M + hy, g.ny, g.periodic_y) * g.nx +
            ghost_index(x0 - M + hx, g.nx, g.periodic_x);
  }
  double qe[2 * M + 1], qp[2 * M + 1];             // planes z - M .. z + M of this column
#pragma unroll
  for (int k = 0; k <= 2 * M; ++k) {
    const size_t o = (size_t)ghost_index(z0 - M + k, g.nz, g.periodic_z) * plane + cxy;
    qe[k] = lne[o];
    qp[k] = phi[o];
  }
  double he[HS], hp[HS];
#pragma unroll
  for (int s = 0; s < HS; ++s) {
    he[s] = lne[(size_t)z0 * plane + ho[s]];
    hp[s] = phi[(size_t)z0 * plane + ho[s]];
  }
  const double scale = AV ? 1.0 / (g.h * g.h) : 1.0 / (4.0 * kPi * g.h * g.h);
  const bool inside = X < g.nx && Y < g.ny;
  double vr = 0.0, vav = 0.0;
  for (int z = z0; z < z1; ++z) {
    te[(M + ty) * TW + M + tx] = qe[M];
    tp[(M + ty) * TW + M + tx] = qp[M];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
      te[hl[s]] = he[s];
      tp[hl[s]] = hp[s];
    }
    __syncthreads();
    const int zn = min(z + 1, g.nz - 1);
    double hne[HS], hnp[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
      hne[s] = lne[(size_t)zn * plane + ho[s]];
      hnp[s] = phi[(size_t)zn * plane + ho[s]];
    }
    const size_t on = (size_t)ghost_index(z + 1 + M, g.nz, g.periodic_z) * plane + cxy;
    const double qne = lne[on], qnp = phi[on];
    double rv = 0.0, ev = 1.0;
    const size_t o = (size_t)z * plane + (size_t)Y * g.nx + X;
    if (inside) {
      rv = rho[o];
      ev = eps[o];
    }
    const double* ce = &te[(M + ty) * TW + M + tx];
    const double* cp = &tp[(M + ty) * TW + M + tx];
    double exd = 0.0, eyd = 0.0, ezd = 0.0, pxd = 0.0, pyd = 0.0, pzd = 0.0;
#pragma unroll
    for (int m = 1; m <= M; ++m) {
      exd = fma(w.c[m], ce[m] - ce[-m], exd);
      eyd = fma(w.c[m], ce[m * TW] - ce[-m * TW], eyd);
      ezd = fma(w.c[m], qe[M + m] - qe[M - m], ezd);
      pxd = fma(w.c[m], cp[m] - cp[-m], pxd);
      pyd = fma(w.c[m], cp[m * TW] - cp[-m * TW], pyd);
      pzd = fma(w.c[m], qp[M + m] - qp[M - m], pzd);
    }
    if (inside) {
      const double dot = (exd * pxd + eyd * pyd + ezd * pzd) * scale;
      if constexpr (AV) {
        const double av = -4.0 * kPi * rv + ev * dot;
        out[o] = av;
        const double aw = paper ? cp[0] : av / (ev * ev);
        vr += aw * rv;
        vav += aw * av;
      } else {
        out[o] = dot - (1.0 - 1.0 / ev) * rv;
      }
    }
    __syncthreads();                              // tile reads done before the next writes
#pragma unroll
    for (int k = 0; k < 2 * M; ++k) {
      qe[k] = qe[k + 1];
      qp[k] = qp[k + 1];
    }
    qe[2 * M] = qne;
    qp[2 * M] = qnp;
#pragma unroll
    for (int s = 0; s < HS; ++s) {
      he[s] = hne[s];
      hp[s] = hnp[s];
    }
  }
  if constexpr (AV) {
    vr = block_sum(vr);
    vav = block_sum(vav);
    if (tid == 0) {
      part[2 * (blockIdx.x - d0)] = vr;
      part[2 * (blockIdx.x - d0) + 1] = vav;
    }
  }
}

static FdFirst fd_first_weights(int M) {
  FdFirst w{};
  double fM = 1.0;
  for (int i = 2; i <= M; ++i) fM *= i;
  for (int m = 1; m <= M; ++m) {
    double fa = 1.0, fb = 1.0;
    for (int i = 2; i <= M - m; ++i) fa *= i;
    for (int i = 2; i <= M + m; ++i) fb *= i;
    w.c[m] = (m % 2 == 1 ? 1.0 : -1.0) * fM * fM / (double(m) * fa * fb);
  }
  return w;
}

static int polarization_zlen(const Geom& g) {
  return stencil_zlen((long long)((g.nx + kPTX - 1) / kPTX) * ((g.ny + kPTY - 1) / kPTY), g.nz);
}

int polarization_groups(const Geom& g) {
  const int zlen = polarization_zlen(g);
  return ((g.nx + kPTX - 1) / kPTX) * ((g.ny + kPTY - 1) / kPTY) * ((g.nz + zlen - 1) / zlen);
}

// lne = ln eps, pointwise
__global__ __launch_bounds__(kThreads) void k_log_field(long long n, const double* __restrict__ eps,
                                                        double* __restrict__ lne) {
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) lne[i] = log(eps[i]);
}

// ---------------------------------------------------------------------------
// Polarization charge without allocation: the ln eps field lives in a
// file-scope device array of kNoAllocMaxPoints doubles (32 MiB), one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel (in host code it is only a stand-in for the symbol); it uses the
// device address that hipGetSymbolAddress returns, looked up once per device
// with that device current.  Every call on a GPU shares that GPU's array:
// calls that overlap on one GPU race on it.  ln eps is written in full before
// it is read, so nothing has to start at zero.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kNoAllocMaxPoints];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

void launch_log_field(long long n, const double* eps, double* lne, hipStream_t s) {
  GPS_LAUNCH(k_log_field, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
             n, eps, lne);
}

template <bool AV>
static void launch_graddot(const Geom& g, int fd_half, int paper, const double* rho,
                           const double* eps, const double* lne, const double* phi, double* out,
                           double* part, const int* stop, const ScDecide& dec, hipStream_t s) {
  const int ntx = (g.nx + kPTX - 1) / kPTX, nty = (g.ny + kPTY - 1) / kPTY;
  const int zlen = polarization_zlen(g);
  const dim3 grid(polarization_groups(g) + (dec.st ? 1 : 0));
  const FdFirst w = fd_first_weights(fd_half);
#define GPS_PF(MM)                                                                        \
  case MM:                                                                                \
    GPS_LAUNCH((k_polarization<MM, AV>), grid, dim3(kPThreads), 0, s, g, w, ntx, nty,     \
               zlen, paper, stop, rho, eps, lne, phi, out, part, dec);                     \
    break;
  switch (fd_half) {
    GPS_PF(1) GPS_PF(2) GPS_PF(3) GPS_PF(4) GPS_PF(5) GPS_PF(6) GPS_PF(7) GPS_PF(8)
    default: break;
  }
#undef GPS_PF
}

void launch_polarization(const Geom& g, int fd_half, const double* rho, const double* eps,
                         const double* lne, const double* phi, double* out, hipStream_t s) {
  launch_graddot<false>(g, fd_half, 0, rho, eps, lne, phi, out, nullptr, nullptr, ScDecide{},
                        s);
}

void launch_sc_operator(const Geom& g, int fd_half, int paper_step, const double* r,
                        const double* eps, const double* lne, const double* v, double* av,
                        double* part, const int* stop, const ScDecide& dec, hipStream_t s) {
  launch_graddot<true>(g, fd_half, paper_step, r, eps, lne, v, av, part, stop, dec, s);
}

// ---------------------------------------------------------------------------
// Pointwise steps and decisions of Algorithm SC / PSD (FP64), device-resident:
// the host only replays captured iterations and polls the state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_sc_begin(long long n, const double* __restrict__ rho,
                                                       const double* __restrict__ eps,
                                                       double* __restrict__ r,
                                                       double* __restrict__ f,
                                                       double* __restrict__ phi,
                                                       double* __restrict__ eps_c,
                                                       double* __restrict__ lne,
                                                       double* __restrict__ part) {
  const long long base = (long long)blockIdx.x * kThreads * kVec + threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) {
      const double ev = eps[i];
      const double ri = -4.0 * kPi * rho[i];
      const double fi = ri / ev;
      r[i] = ri;
      f[i] = fi;
      phi[i] = 0.0;
      eps_c[i] = ev;
      lne[i] = log(ev);
      a0 += ri * ri;
      a1 += fi * fi;
    }
  }
  a0 = block_sum(a0);
  a1 = block_sum(a1);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a0;
    part[2 * blockIdx.x + 1] = a1;
  }
}

__global__ __launch_bounds__(kThreads) void k_sc_start(const double* __restrict__ part, int nparts,
                                                       ScState* st, int method, double eta,
                                                       double tol, int max_steps) {
  const double rr0 = sum_partials(part, nparts, 2);
  const double ff0 = sum_partials(part + 1, nparts, 2);
  if (threadIdx.x == 0) {
    ScState z{};
    z.method = method;
    z.eta = eta;
    z.max_steps = max_steps;
    z.status = GPS_E_NOT_CONVERGED;
    z.rr0 = rr0;
    z.rr = rr0;
    z.ff = ff0;
    z.ff_prev = ff0;
    z.thr_w = tol * sqrt(ff0);
    z.thr_r = tol * sqrt(rr0);
    z.thr_sc = tol * sqrt(rr0) / kFourPi;
    if (!isfinite(rr0) || !isfinite(ff0)) {
      z.status = GPS_E_NONFINITE;
      z.done = 1;
    } else if (rr0 == 0.0 || max_steps < 1) {
      z.status = rr0 == 0.0 ? GPS_OK : GPS_E_NOT_CONVERGED;
      z.done = 1;
    }
    *st = z;
  }
}

__global__ __launch_bounds__(kThreads) void k_sc_update(long long n, const double* __restrict__ eps,
                                                        double* __restrict__ phi,
                                                        double* __restrict__ r,
                                                        const double* __restrict__ v,
                                                        const double* __restrict__ av,
                                                        double* __restrict__ f,
                                                        const double* __restrict__ op_part,
                                                        int n_op, double* __restrict__ part,
                                                        ScState* st) {
  if (st->done) return;
  // alpha, identical in every work-group (fixed-order sums of the operator's partials)
  const double vr = sum_partials(op_part, n_op, 2);
  const double vav = sum_partials(op_part + 1, n_op, 2);
  const int method = st->method;
  double alpha;
  int fail = 0;
  if (method == GPS_METHOD_SC) {
    alpha = (st->step == 0 ? -1.0 : -st->eta) / kFourPi;
  } else {
    if (!isfinite(vr) || !isfinite(vav)) fail = GPS_E_NONFINITE;
    else if (method == GPS_METHOD_PSD ? vav == 0.0 : !(vav > 0.0)) fail = GPS_E_BREAKDOWN;
    alpha = fail ? 0.0 : vr / vav;
  }
  if (fail) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {   // the decision ends the solve
      st->status = fail;
      st->pending = 1;
    }
    return;
  }
  const long long base = (long long)blockIdx.x * kThreads * kVec + threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) {
      phi[i] += alpha * v[i];
      const double ri = r[i] - alpha * av[i];
      const double fi = ri / eps[i];
      r[i] = ri;
      f[i] = fi;
      a0 += ri * ri;
      a1 += fi * fi;
    }
  }
  a0 = block_sum(a0);
  a1 = block_sum(a1);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a0;
    part[2 * blockIdx.x + 1] = a1;
    if (blockIdx.x == 0) {
      st->alpha = alpha;
      st->pending = 1;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_sc_decide(ScDecide dec) {
  sc_decide_group(dec.part, dec.nparts, dec.st);
}

__global__ __launch_bounds__(kThreads) void k_sc_energy(long long n, const double* __restrict__ rho,
                                                        const double* __restrict__ phi,
                                                        double* __restrict__ part) {
  const long long base = (long long)blockIdx.x * kThreads * kVec + threadIdx.x;
  double a0 = 0.0;
#pragma unroll
  for (int j = 0; j < kVec; ++j) {
    const long long i = base + (long long)j * kThreads;
    if (i < n) a0 += rho[i] * phi[i];
  }
  a0 = block_sum(a0);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a0;
    part[2 * blockIdx.x + 1] = 0.0;
  }
}

void launch_sc_begin(long long n, const double* rho, const double* eps, double* r, double* f,
                     double* phi, double* eps_c, double* lne, double* part, ScState* st,
                     int method, double eta, double tol, int max_steps, hipStream_t s) {
  const int gv = vec_groups(n);
  GPS_LAUNCH(k_sc_begin, dim3(gv), dim3(kThreads), 0, s, n, rho, eps, r, f, phi, eps_c, lne,
             part);
  GPS_LAUNCH(k_sc_start, dim3(1), dim3(kThreads), 0, s, part, gv, st, method, eta, tol,
             max_steps);
}

void launch_sc_advance(long long n, const double* eps, double* phi, double* r, const double* v,
                       const double* av, double* f, const double* op_part, int n_op,
                       double* part, ScState* st, hipStream_t s) {
  const int gv = vec_groups(n);
  GPS_LAUNCH(k_sc_update, dim3(gv), dim3(kThreads), 0, s, n, eps, phi, r, v, av, f, op_part,
             n_op, part, st);
}

void launch_sc_decide(const ScDecide& dec, hipStream_t s) {
  GPS_LAUNCH(k_sc_decide, dim3(1), dim3(kThreads), 0, s, dec);
}

void launch_sc_energy(long long n, const double* rho, const double* phi, double* part,
                      hipStream_t s) {
  GPS_LAUNCH(k_sc_energy, dim3(vec_groups(n)), dim3(kThreads), 0, s, n, rho, phi, part);
}

}  // namespace gps
