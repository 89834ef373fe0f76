// Two-level FFT passes for the pencil lengths of the common grids.
//
// A length L = L1 * L2 transform of a tile of pencils runs as
//   forward:  x[L2 n1 + n2] --(L1-point DFT over n1, in registers)--> Y[n2][k1]
//             Y *= w_L^(n2 k1); one exchange through LDS;
//             (L2-point DFT over n2, in registers) --> X[k1 + L1 k2]
//   inverse:  X[k1 + L1 k2] --(L2-point inverse DFT over k2)--> Z[k1][n_a]
//             Z *= w_L^(-n_a k1); one exchange through LDS;
//             (L1-point inverse DFT over k1) --> x[n_a + L2 n_b]
// so a pass touches LDS once per direction instead of once per radix stage.
// The z pass keeps the spectrum in registers between the forward transform,
// the multiplication by the Green's spectrum and the inverse transform.
//
// Strided (y, z) passes load and store directly between HBM and registers:
// a thread owns one column of one pencil, threads of a wavefront cover B
// adjacent pencils, so every row access is a contiguous B-element segment.
// The x passes stage rows through LDS to keep their loads and stores
// contiguous along x.
#include "gps_fft_reg.h"
#include "gps_iter.h"
#include "gps_launch.h"

namespace gps {

template <typename T> struct FastTile;
template <> struct FastTile<float> { static constexpr int B = 16; };
template <> struct FastTile<double> { static constexpr int B = 8; };
constexpr int kXPairs = 4;             // row pairs per work-group of the x passes

constexpr int round64(int v) { return (v + 63) / 64 * 64; }

template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return cmk(a.x, -a.y); }

// ---------------------------------------------------------------------------
// strided passes
// ---------------------------------------------------------------------------
template <typename T, int L1, int L2, int MODE>
__global__ __launch_bounds__(round64(FastTile<T>::B * L1))
void k_fstrided(SParams<T> p) {
  constexpr int B = FastTile<T>::B;
  constexpr int L = L1 * L2;
  constexpr int PITCH = B + 1;
  __shared__ cplx<T> lds[L * PITCH];
  const int tid = threadIdx.x;
  cplx<T>* work = p.work;
  double g0 = 0.0;
  if (work == nullptr) {
    const Slot<T>& sl = p.slots[p.batch.slot[blockIdx.y]];
    if (wg_read_flag(&sl.st->done)) return;
    work = sl.work;
    g0 = sl.g0;
  }
  const int b = tid & (B - 1);
  const int q = tid / B;
  const int pen = xcd_tile(blockIdx.x, gridDim.x) * B + b;
  const bool pv = pen < p.npencils;
  size_t base = 0;
  if (pv) {
    const int grp = pen / p.per_group;
    base = (size_t)grp * p.group_stride + (pen - grp * p.per_group);
  }
  const size_t es = (size_t)p.elem_stride;
  const cplx<T>* __restrict__ tw = p.tw;

  cplx<T> y[L2];
  if constexpr (MODE != ST_INV) {
    if (q < L2) {
      cplx<T> x[L1];
#pragma unroll
      for (int n1 = 0; n1 < L1; ++n1) {
        const int t = L2 * n1 + q;
        x[n1] = (pv && t < p.Lin) ? work[base + t * es] : cmk(T(0), T(0));
      }
      reg_fft<T, false, L1>(x);
#pragma unroll
      for (int k1 = 1; k1 < L1; ++k1) x[k1] = cmul(x[k1], tw[q * k1]);
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) lds[(q * L1 + k1) * PITCH + b] = x[k1];
    }
    __syncthreads();
    if (q < L1) {
#pragma unroll
      for (int n2 = 0; n2 < L2; ++n2) y[n2] = lds[(n2 * L1 + q) * PITCH + b];
      reg_fft<T, false, L2>(y);                 // y[k2] = X[q + L1 k2]
    }
    if constexpr (MODE == ST_FWD) {
      if (pv && q < L1) {
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) {
          const int kk = q + L1 * k2;
          if (kk < p.Lout) work[base + kk * es] = y[k2];
        }
      }
      return;
    } else {
      if (pv && q < L1) {
        const int Lyh = p.Ly / 2 + 1;
        const int ky = pen / p.Kx;
        const int kx = pen - ky * p.Kx;
        const int kyf = min(ky, p.Ly - ky);
        const T* __restrict__ row = p.table + (size_t)kyf * p.Kx + kx;
        const size_t zs = (size_t)Lyh * p.Kx;
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) {
          const int kz = q + L1 * k2;
          const int kzf = min(kz, L - kz);
          T m = row[kzf * zs];
          if (p.k0_from_slot && pen == 0 && kz == 0) m = T(g0);
          y[k2] = cscale(y[k2], m);
        }
      }
      __syncthreads();                          // step-2 reads of lds are done
    }
  } else {
    if (q < L1) {
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) {
        const int kk = q + L1 * k2;
        y[k2] = (pv && kk < p.Lin) ? work[base + kk * es] : cmk(T(0), T(0));
      }
    }
  }
  // inverse transform (ST_CONV second half, ST_INV)
  if (q < L1) {
    reg_fft<T, true, L2>(y);                    // y[n_a] = Z[q][n_a]
#pragma unroll
    for (int na = 1; na < L2; ++na) y[na] = cmul(y[na], cconj(tw[na * q]));
#pragma unroll
    for (int na = 0; na < L2; ++na) lds[(na * L1 + q) * PITCH + b] = y[na];
  }
  __syncthreads();
  if (q < L2) {
    cplx<T> x[L1];
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) x[k1] = lds[(q * L1 + k1) * PITCH + b];
    reg_fft<T, true, L1>(x);                    // x[n_b] = out[q + L2 n_b]
    if (pv) {
#pragma unroll
      for (int nb = 0; nb < L1; ++nb) {
        const int t = q + L2 * nb;
        if (t < p.Lout) work[base + t * es] = x[nb];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// x passes (pairs of real rows packed as one complex row)
// ---------------------------------------------------------------------------
template <typename T, int L1, int L2, int MODE>
__global__ __launch_bounds__(round64(kXPairs * L1))
void k_fxfwd(XParams<T> p) {
  constexpr int P = kXPairs;
  constexpr int L = L1 * L2;
  constexpr int PITCH = P + 1;
  __shared__ cplx<T> lds[L * PITCH];
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int Kx = p.g.Kx, Lin = p.Lin;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int pair0 = tile * P;
  cplx<T>* work = p.work;
  Slot<T> sl;
  double alpha = 0.0;
  bool upd = false;
  if constexpr (MODE == XF_SOLVE) {
    sl = p.slots[p.batch.slot[blockIdx.y]];
    int k;
    if (!xfwd_head(sl, p.n_vec_parts, &k, &alpha)) return;
    upd = k > 0;
    work = sl.work;
  }
  double mu = 0.0;
  for (int e = tid; e < P * Lin; e += nt) {
    const int pp = e / Lin;
    const int x = e - pp * Lin;
    const int ra = 2 * (pair0 + pp), rb = ra + 1;
    T a = T(0), bb = T(0);
    if constexpr (MODE == XF_SOLVE) {
      if (ra < p.nrows) a = solve_prologue(sl, (size_t)ra * p.in_row_stride + x, upd, alpha);
      if (rb < p.nrows) bb = solve_prologue(sl, (size_t)rb * p.in_row_stride + x, upd, alpha);
      mu += double(a) + double(bb);
    } else {
      if (ra < p.nrows) a = T(p.in_real[(size_t)ra * p.in_row_stride + x]);
      if (rb < p.nrows) bb = T(p.in_real[(size_t)rb * p.in_row_stride + x]);
    }
    lds[x * PITCH + pp] = cmk(a, bb);
  }
  for (int e = tid; e < P * (L - Lin); e += nt) {
    const int x = Lin + e / P;
    lds[x * PITCH + (e % P)] = cmk(T(0), T(0));
  }
  __syncthreads();
  const int pp = tid % P;
  const int q = tid / P;
  const cplx<T>* __restrict__ tw = p.tw;
  cplx<T> x[L1];
  if (q < L2) {
#pragma unroll
    for (int n1 = 0; n1 < L1; ++n1) x[n1] = lds[(L2 * n1 + q) * PITCH + pp];
    reg_fft<T, false, L1>(x);
#pragma unroll
    for (int k1 = 1; k1 < L1; ++k1) x[k1] = cmul(x[k1], tw[q * k1]);
  }
  __syncthreads();
  if (q < L2) {
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) lds[(q * L1 + k1) * PITCH + pp] = x[k1];
  }
  __syncthreads();
  cplx<T> y[L2];
  if (q < L1) {
#pragma unroll
    for (int n2 = 0; n2 < L2; ++n2) y[n2] = lds[(n2 * L1 + q) * PITCH + pp];
    reg_fft<T, false, L2>(y);
  }
  __syncthreads();
  if (q < L1) {
#pragma unroll
    for (int k2 = 0; k2 < L2; ++k2) lds[(q + L1 * k2) * PITCH + pp] = y[k2];
  }
  __syncthreads();
  for (int e = tid; e < P * Kx; e += nt) {
    const int p2 = e / Kx;
    const int kk = e - p2 * Kx;
    const int ra = 2 * (pair0 + p2), rb = ra + 1;
    const cplx<T> zk = lds[kk * PITCH + p2];
    const int km = kk == 0 ? 0 : L - kk;
    const cplx<T> zm = lds[km * PITCH + p2];
    const T half = T(0.5);
    const cplx<T> xa = cmk(half * (zk.x + zm.x), half * (zk.y - zm.y));
    const cplx<T> xb = cmk(half * (zk.y + zm.y), half * (zm.x - zk.x));
    if (ra < p.nrows)
      work[(size_t)(ra / p.rows_per_plane) * p.plane_stride +
           (size_t)(ra % p.rows_per_plane) * Kx + kk] = xa;
    if (rb < p.nrows)
      work[(size_t)(rb / p.rows_per_plane) * p.plane_stride +
           (size_t)(rb % p.rows_per_plane) * Kx + kk] = xb;
  }
  if constexpr (MODE == XF_SOLVE) {
    if (p.periodic_mean) {
      const double s = block_sum(mu);
      if (tid == 0) sl.part_mu[tile] = s;
    }
  }
}

template <typename T, int L1, int L2, int MODE>   // MODE 0: solve epilogue, 1: plain store
__global__ __launch_bounds__(round64(kXPairs * L1))
void k_fxinv(XParams<T> p) {
  constexpr int P = kXPairs;
  constexpr int L = L1 * L2;
  constexpr int PITCH = P + 1;
  __shared__ cplx<T> lds[L * PITCH];
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int Kx = p.g.Kx, Lout = p.Lout;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int pair0 = tile * P;
  cplx<T>* work = p.work;
  Slot<T> sl;
  if constexpr (MODE == 0) {
    sl = p.slots[p.batch.slot[blockIdx.y]];
    if (wg_read_flag(&sl.st->done)) return;
    work = sl.work;
  }
  for (int e = tid; e < P * Kx; e += nt) {
    const int p2 = e / Kx;
    const int kk = e - p2 * Kx;
    const int ra = 2 * (pair0 + p2), rb = ra + 1;
    cplx<T> xa = cmk(T(0), T(0)), xb = cmk(T(0), T(0));
    if (ra < p.nrows)
      xa = work[(size_t)(ra / p.rows_per_plane) * p.plane_stride +
                (size_t)(ra % p.rows_per_plane) * Kx + kk];
    if (rb < p.nrows)
      xb = work[(size_t)(rb / p.rows_per_plane) * p.plane_stride +
                (size_t)(rb % p.rows_per_plane) * Kx + kk];
    if (kk == 0 || 2 * kk == L) {
      xa.y = T(0);
      xb.y = T(0);
    }
    lds[kk * PITCH + p2] = cmk(xa.x - xb.y, xa.y + xb.x);
    const int km = L - kk;
    if (kk > 0 && km >= Kx) lds[km * PITCH + p2] = cmk(xa.x + xb.y, xb.x - xa.y);
  }
  __syncthreads();
  const int pp = tid % P;
  const int q = tid / P;
  const cplx<T>* __restrict__ tw = p.tw;
  cplx<T> y[L2];
  if (q < L1) {
#pragma unroll
    for (int k2 = 0; k2 < L2; ++k2) y[k2] = lds[(q + L1 * k2) * PITCH + pp];
    reg_fft<T, true, L2>(y);
#pragma unroll
    for (int na = 1; na < L2; ++na) y[na] = cmul(y[na], cconj(tw[na * q]));
  }
  __syncthreads();
  if (q < L1) {
#pragma unroll
    for (int na = 0; na < L2; ++na) lds[(na * L1 + q) * PITCH + pp] = y[na];
  }
  __syncthreads();
  cplx<T> x[L1];
  if (q < L2) {
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) x[k1] = lds[(q * L1 + k1) * PITCH + pp];
    reg_fft<T, true, L1>(x);
  }
  __syncthreads();
  if (q < L2) {
#pragma unroll
    for (int nb = 0; nb < L1; ++nb) lds[(q + L2 * nb) * PITCH + pp] = x[nb];
  }
  __syncthreads();
  double acc = 0.0, acc2 = 0.0;
  for (int e = tid; e < P * Lout; e += nt) {
    const int p2 = e / Lout;
    const int xx = e - p2 * Lout;
    const int ra = 2 * (pair0 + p2), rb = ra + 1;
    const cplx<T> z = lds[xx * PITCH + p2];
    if (ra < p.nrows) {
      const size_t o = (size_t)ra * p.in_row_stride + xx;
      if constexpr (MODE == 0) solve_epilogue(sl, o, z.x, acc, acc2);
      else p.out_real[o] = double(z.x);
    }
    if (rb < p.nrows) {
      const size_t o = (size_t)rb * p.in_row_stride + xx;
      if constexpr (MODE == 0) solve_epilogue(sl, o, z.y, acc, acc2);
      else p.out_real[o] = double(z.y);
    }
  }
  if constexpr (MODE == 0) {
    const double s1 = block_sum(acc);
    const double s2 = block_sum(acc2);
    if (tid == 0) {
      sl.part_delta[0][tile] = s1;
      sl.part_rr[tile] = s2;
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define GPS_FAST_LENGTHS(X) \
  X(32, 8, 4) X(48, 8, 6) X(64, 8, 8) X(96, 12, 8) X(128, 16, 8) X(192, 16, 12) \
  X(256, 16, 16) X(320, 20, 16) X(384, 24, 16)

bool fast_length(int L) {
  switch (L) {
#define GPS_CASE(LL, A, B) case LL: return true;
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
    default: return false;
  }
}

int fast_xpass_groups(int nrows) { return ((nrows + 1) / 2 + kXPairs - 1) / kXPairs; }

template <typename T>
bool fast_strided(int mode, const SParams<T>& p, hipStream_t s) {
  constexpr int B = FastTile<T>::B;
  const dim3 grid((p.npencils + B - 1) / B, p.work ? 1 : p.batch.n);
  switch (p.L) {
#define GPS_CASE(LL, A, BB)                                                                    \
  case LL: {                                                                                   \
    const dim3 blk(round64(B * A));                                                            \
    if (mode == ST_FWD) hipLaunchKernelGGL((k_fstrided<T, A, BB, ST_FWD>), grid, blk, 0, s, p);  \
    else if (mode == ST_INV) hipLaunchKernelGGL((k_fstrided<T, A, BB, ST_INV>), grid, blk, 0, s, p); \
    else hipLaunchKernelGGL((k_fstrided<T, A, BB, ST_CONV>), grid, blk, 0, s, p);             \
    return true;                                                                               \
  }
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
    default: return false;
  }
}

template <typename T>
bool fast_xfwd(int mode, const XParams<T>& p, hipStream_t s) {
  if (mode != XF_SOLVE && mode != XF_REAL) return false;
  const dim3 grid(fast_xpass_groups(p.nrows), p.slots ? p.batch.n : 1);
  switch (p.g.Lx) {
#define GPS_CASE(LL, A, BB)                                                                    \
  case LL: {                                                                                   \
    const dim3 blk(round64(kXPairs * A));                                                      \
    if (mode == XF_SOLVE) hipLaunchKernelGGL((k_fxfwd<T, A, BB, XF_SOLVE>), grid, blk, 0, s, p); \
    else hipLaunchKernelGGL((k_fxfwd<T, A, BB, XF_REAL>), grid, blk, 0, s, p);                \
    return true;                                                                               \
  }
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
    default: return false;
  }
}

template <typename T>
bool fast_xinv(int mode, const XParams<T>& p, hipStream_t s) {
  const dim3 grid(fast_xpass_groups(p.nrows), p.slots ? p.batch.n : 1);
  switch (p.g.Lx) {
#define GPS_CASE(LL, A, BB)                                                                    \
  case LL: {                                                                                   \
    const dim3 blk(round64(kXPairs * A));                                                      \
    if (mode == 0) hipLaunchKernelGGL((k_fxinv<T, A, BB, 0>), grid, blk, 0, s, p);            \
    else hipLaunchKernelGGL((k_fxinv<T, A, BB, 1>), grid, blk, 0, s, p);                      \
    return true;                                                                               \
  }
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
    default: return false;
  }
}

template bool fast_strided<float>(int, const SParams<float>&, hipStream_t);
template bool fast_strided<double>(int, const SParams<double>&, hipStream_t);
template bool fast_xfwd<float>(int, const XParams<float>&, hipStream_t);
template bool fast_xfwd<double>(int, const XParams<double>&, hipStream_t);
template bool fast_xinv<float>(int, const XParams<float>&, hipStream_t);
template bool fast_xinv<double>(int, const XParams<double>&, hipStream_t);

}  // namespace gps
