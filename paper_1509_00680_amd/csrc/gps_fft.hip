// FFT passes of the vacuum Poisson solver used as PCG preconditioner
// (Eq. PCGdef: v = S^-1 G S^-1 r, G a zero-padded FFT convolution).
//
// Every pass keeps one tile of pencils in LDS and runs a self-sorting
// (Stockham) mixed-radix FFT on it.  Tiles hold B adjacent pencils with the
// pencil index fastest, so global loads and stores of a tile row are
// contiguous.  Zero padding is pruned: the zero half of a padded axis is
// never read from or written to HBM.
//
//   x pass   two real rows packed as one complex row (R2C / C2R pairing);
//            fused prologue r/sqrt(eps) and epilogue u/sqrt(eps) + (v, r).
//   y pass   strided C2C, in place in the work buffer.
//   z pass   strided C2C forward, multiply by the real even Green's
//            spectrum, C2C inverse, all in one pass through LDS.
#include "gps_iter.h"
#include "gps_launch.h"

namespace gps {

// ---------------------------------------------------------------------------
// small DFTs
// ---------------------------------------------------------------------------
template <int R> struct Roots;
template <> struct Roots<3> {
  static constexpr double c[2] = {1.0, -0.5};
  static constexpr double s[2] = {0.0, 0.86602540378443864676};
};
template <> struct Roots<5> {
  static constexpr double c[3] = {1.0, 0.30901699437494742410, -0.80901699437494742410};
  static constexpr double s[3] = {0.0, 0.95105651629515357212, 0.58778525229247312917};
};
template <> struct Roots<7> {
  static constexpr double c[4] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                  -0.90096886790241912624};
  static constexpr double s[4] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                  0.43388373911755812048};
};

// y_k = sum_n x_n w^(nk), w = exp(-2 pi i/R) (forward) or its conjugate.
template <typename T, bool INV, int R>
__device__ __forceinline__ void dft(cplx<T>* x) {
  if constexpr (R == 2) {
    cplx<T> a = x[0];
    x[0] = cadd(a, x[1]);
    x[1] = csub(a, x[1]);
  } else if constexpr (R == 4) {
    cplx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    cplx<T> a2 = cadd(x[1], x[3]), a3 = csub(x[1], x[3]);
    // forward: (-i) a3 ; inverse: (+i) a3
    cplx<T> ja3 = INV ? cmk(-a3.y, a3.x) : cmk(a3.y, -a3.x);
    x[0] = cadd(a0, a2);
    x[2] = csub(a0, a2);
    x[1] = cadd(a1, ja3);
    x[3] = csub(a1, ja3);
  } else {
    constexpr int H = (R - 1) / 2;
    cplx<T> a[H + 1], b[H + 1];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      a[n] = cadd(x[n], x[R - n]);
      b[n] = csub(x[n], x[R - n]);
    }
    cplx<T> x0 = x[0];
    cplx<T> y0 = x0;
#pragma unroll
    for (int n = 1; n <= H; ++n) y0 = cadd(y0, a[n]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cplx<T> re = x0, im = cmk(T(0), T(0));
#pragma unroll
      for (int n = 1; n <= H; ++n) {
        const int m = (n * k) % R;
        const int mf = m <= H ? m : R - m;
        const T cs = T(Roots<R>::c[mf]);
        const T sn = T(m <= H ? Roots<R>::s[mf] : -Roots<R>::s[mf]);
        re = cadd(re, cscale(a[n], cs));
        im = cadd(im, cscale(b[n], sn));
      }
      // y_k = re - i im (forward), y_{R-k} = re + i im
      cplx<T> mi = cmk(im.y, -im.x);   // -i * im
      if (INV) {
        x[k] = csub(re, mi);
        x[R - k] = cadd(re, mi);
      } else {
        x[k] = cadd(re, mi);
        x[R - k] = csub(re, mi);
      }
    }
    x[0] = y0;
  }
}

// One Stockham stage of radix R over a tile of B = 2^lgB pencils of length L
// stored as buf[t * B + b].  Ns = product of the radices of earlier stages.
template <typename T, bool INV, int R>
__device__ __forceinline__ void stage(cplx<T>* __restrict__ buf, int L, int lgB, int Ns,
                                      const cplx<T>* __restrict__ tw) {
  constexpr int MAXE = TileCap<T>::elems;
  constexpr int MAXBF = (MAXE + R * kThreads - 1) / (R * kThreads);
  const int B = 1 << lgB;
  const int LR = L / R;
  const int nbf = LR << lgB;
  const int twstride = L / (Ns * R);
  const int tid = threadIdx.x;
  cplx<T> x[MAXBF][R];
#pragma unroll
  for (int i = 0; i < MAXBF; ++i) {
    const int e = tid + i * kThreads;
    if (e < nbf) {
      const int b = e & (B - 1);
      const int j = e >> lgB;
#pragma unroll
      for (int r = 0; r < R; ++r) x[i][r] = buf[((j + r * LR) << lgB) + b];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXBF; ++i) {
    const int e = tid + i * kThreads;
    if (e < nbf) {
      const int b = e & (B - 1);
      const int j = e >> lgB;
      const int jq = j / Ns;
      const int k = j - jq * Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cplx<T> w = tw[r * k * twstride];
        if (INV) w.y = -w.y;
        x[i][r] = cmul(x[i][r], w);
      }
      dft<T, INV, R>(x[i]);
      const int base = jq * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[((base + r * Ns) << lgB) + b] = x[i][r];
    }
  }
  __syncthreads();
}

template <typename T, bool INV>
__device__ void lds_fft(cplx<T>* buf, int L, int lgB, const RadixPlan& rp,
                        const cplx<T>* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < rp.nstages; ++s) {
    const int R = rp.radix[s];
    switch (R) {
      case 4: stage<T, INV, 4>(buf, L, lgB, Ns, tw); break;
      case 2: stage<T, INV, 2>(buf, L, lgB, Ns, tw); break;
      case 3: stage<T, INV, 3>(buf, L, lgB, Ns, tw); break;
      case 5: stage<T, INV, 5>(buf, L, lgB, Ns, tw); break;
      default: stage<T, INV, 7>(buf, L, lgB, Ns, tw); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------
// cell-averaged 1/r (free-boundary Green's function, plan time, FP64)
// ---------------------------------------------------------------------------
// F with d^3F/dxdydz = 1/|r| (x, y, z nonzero).
__device__ double prism_antiderivative(double x, double y, double z) {
  const double r = sqrt(x * x + y * y + z * z);
  return y * z * log(x + r) + x * z * log(y + r) + x * y * log(z + r)
         - 0.5 * x * x * atan(y * z / (x * r)) - 0.5 * y * y * atan(x * z / (y * r))
         - 0.5 * z * z * atan(x * y / (z * r));
}

// Integral of 1/|u| over the unit cube centred at (mx, my, mz), mx, my, mz >= 0.
// Exact through the 8 corners for max(m) <= 8; beyond, 1/r plus the r^-5 and
// r^-7 terms of the cube average sinh(d/2)/(d/2) applied to the harmonic 1/r.
__device__ double cell_inverse_distance(int mx, int my, int mz) {
  const int mmax = max(mx, max(my, mz));
  if (mmax <= 8) {
    double s = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
      const double f = prism_antiderivative(mx - 0.5 + sx, my - 0.5 + sy, mz - 0.5 + sz);
      s += ((sx + sy + sz) & 1) ? f : -f;
    }
    return s;
  }
  const double x2 = double(mx) * mx, y2 = double(my) * my, z2 = double(mz) * mz;
  const double r2 = x2 + y2 + z2;
  const double r = sqrt(r2);
  const double s4 = x2 * x2 + y2 * y2 + z2 * z2;
  const double p22 = x2 * y2 + x2 * z2 + y2 * z2;
  const double r4 = r2 * r2;
  const double t4 = (-7.0 / 480.0 * s4 + 7.0 / 160.0 * p22) / (r4 * r4 * r);
  const double s6 = x2 * x2 * x2 + y2 * y2 * y2 + z2 * z2 * z2;
  const double p42 = x2 * x2 * (y2 + z2) + y2 * y2 * (x2 + z2) + z2 * z2 * (x2 + y2);
  const double r12 = r4 * r4 * r4;
  const double t6 = (2.0 * s6 - 15.0 * p42 + 180.0 * x2 * y2 * z2) / 1344.0 / (r12 * r);
  return 1.0 / r + t4 + t6;
}

// ---------------------------------------------------------------------------
// x passes
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_xfwd(XParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int Lx = p.g.Lx, Kx = p.g.Kx, P = p.P, lgP = p.lgP, Lin = p.Lin;
  const int pair0 = blockIdx.x * P;
  cplx<T>* work = p.work;
  const Slot<T> sl = p.tab.s[p.batch.slot[blockIdx.y]];
  double alpha = 0.0;
  bool upd = false;
  if constexpr (MODE == XF_SOLVE) {
    int k;
    XHead<> hd;
    xfwd_head_load(sl, p.n_pap_parts, hd);
    if (!xfwd_head_finish(sl, p.n_pap_parts, hd, &k, &alpha, &upd)) return;
    work = sl.work;
  }
  double mu = 0.0, rr = 0.0;
  for (int e = tid; e < P * Lin; e += kThreads) {
    const int pp = e / Lin;
    const int x = e - pp * Lin;
    const int ra = 2 * (pair0 + pp), rb = ra + 1;
    T a = T(0), b = T(0);
    if constexpr (MODE == XF_SOLVE) {
      if (ra < p.nrows) a = solve_prologue(sl, (size_t)ra * p.in_row_stride + x, upd, alpha, rr);
      if (rb < p.nrows) b = solve_prologue(sl, (size_t)rb * p.in_row_stride + x, upd, alpha, rr);
      mu += double(a) + double(b);
    } else if constexpr (MODE == XF_REAL) {
      if (ra < p.nrows) a = T(p.in_real[(size_t)ra * p.in_row_stride + x]);
      if (rb < p.nrows) b = T(p.in_real[(size_t)rb * p.in_row_stride + x]);
    } else {   // XF_GEN_FREE: K(m) = I(m)/h on the cyclic padded grid
      const int mx = x <= p.g.nx ? x : Lx - x;
      const double inv_h = 1.0 / p.g.h;
      if (ra < p.nrows) {
        const int y = ra % p.rows_per_plane, z = ra / p.rows_per_plane;
        const int my = y <= p.g.ny ? y : p.g.Ly - y, mz = z <= p.g.nz ? z : p.g.Lz - z;
        a = T(cell_inverse_distance(mx, my, mz) * inv_h);
      }
      if (rb < p.nrows) {
        const int y = rb % p.rows_per_plane, z = rb / p.rows_per_plane;
        const int my = y <= p.g.ny ? y : p.g.Ly - y, mz = z <= p.g.nz ? z : p.g.Lz - z;
        b = T(cell_inverse_distance(mx, my, mz) * inv_h);
      }
    }
    buf[(x << lgP) + pp] = cmk(a, b);
  }
  for (int e = tid; e < P * (Lx - Lin); e += kThreads) {
    buf[((Lin + (e >> lgP)) << lgP) + (e & (P - 1))] = cmk(T(0), T(0));
  }
  __syncthreads();
  lds_fft<T, false>(buf, Lx, lgP, p.rp, p.tw);
  for (int e = tid; e < P * Kx; e += kThreads) {
    const int pp = e / Kx;
    const int kk = e - pp * Kx;
    const int ra = 2 * (pair0 + pp), rb = ra + 1;
    const cplx<T> zk = buf[(kk << lgP) + pp];
    const int km = kk == 0 ? 0 : Lx - kk;
    const cplx<T> zm = buf[(km << lgP) + pp];
    const T half = T(0.5);
    const cplx<T> xa = cmk(half * (zk.x + zm.x), half * (zk.y - zm.y));
    const cplx<T> xb = cmk(half * (zk.y + zm.y), half * (zm.x - zk.x));
    if (ra < p.nrows) {
      const size_t o = (size_t)(ra / p.rows_per_plane) * p.plane_stride +
                       (size_t)(ra % p.rows_per_plane) * Kx + kk;
      work[o] = xa;
    }
    if (rb < p.nrows) {
      const size_t o = (size_t)(rb / p.rows_per_plane) * p.plane_stride +
                       (size_t)(rb % p.rows_per_plane) * Kx + kk;
      work[o] = xb;
    }
  }
  if constexpr (MODE == XF_SOLVE) {
    const double s2 = block_sum(rr);
    if (tid == 0) sl.part_rr[blockIdx.x] = s2;
    if (p.periodic_mean) {
      const double s = block_sum(mu);
      if (tid == 0) sl.part_mu[blockIdx.x] = s;
    }
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_xinv(XParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int Lx = p.g.Lx, Kx = p.g.Kx, P = p.P, lgP = p.lgP, Lout = p.Lout;
  const int pair0 = blockIdx.x * P;
  cplx<T>* work = p.work;
  const Slot<T> sl = p.tab.s[p.batch.slot[blockIdx.y]];
  DirArgs dir{};
  if constexpr (MODE == XI_SOLVE) {
    if (solve_stopped(sl.st)) return;
    work = sl.work;
    dir.fresh = sl.st->fresh;
    dir.beta = sl.st->beta;
    dir.mu = p.periodic_mean ? sl.st->mu : 0.0;
  }
  for (int e = tid; e < P * Kx; e += kThreads) {
    const int pp = e / Kx;
    const int kk = e - pp * Kx;
    const int ra = 2 * (pair0 + pp), rb = ra + 1;
    cplx<T> xa = cmk(T(0), T(0)), xb = cmk(T(0), T(0));
    if (ra < p.nrows)
      xa = work[(size_t)(ra / p.rows_per_plane) * p.plane_stride +
                (size_t)(ra % p.rows_per_plane) * Kx + kk];
    if (rb < p.nrows)
      xb = work[(size_t)(rb / p.rows_per_plane) * p.plane_stride +
                (size_t)(rb % p.rows_per_plane) * Kx + kk];
    if (kk == 0 || 2 * kk == Lx) {   // self-conjugate bins of a real row
      xa.y = T(0);
      xb.y = T(0);
    }
    buf[(kk << lgP) + pp] = cmk(xa.x - xb.y, xa.y + xb.x);          // xa + i xb
    const int km = Lx - kk;
    if (kk > 0 && km >= Kx) buf[(km << lgP) + pp] = cmk(xa.x + xb.y, xb.x - xa.y);
  }
  __syncthreads();
  lds_fft<T, true>(buf, Lx, lgP, p.rp, p.tw);
  const bool per = p.periodic_mean != 0;
  double acc = 0.0;
  for (int e = tid; e < P * Lout; e += kThreads) {
    const int pp = e / Lout;
    const int x = e - pp * Lout;
    const int ra = 2 * (pair0 + pp), rb = ra + 1;
    const cplx<T> z = buf[(x << lgP) + pp];
    if (ra < p.nrows) {
      const size_t o = (size_t)ra * p.in_row_stride + x;
      if constexpr (MODE == XI_SOLVE) solve_epilogue(sl, o, z.x, dir, per, acc);
      else p.out_real[o] = double(z.x);
    }
    if (rb < p.nrows) {
      const size_t o = (size_t)rb * p.in_row_stride + x;
      if constexpr (MODE == XI_SOLVE) solve_epilogue(sl, o, z.y, dir, per, acc);
      else p.out_real[o] = double(z.y);
    }
  }
  if constexpr (MODE == XI_SOLVE) {
    const double s1 = block_sum(acc);
    if (tid == 0) sl.part_pap[blockIdx.x] = s1;
  }
}

// ---------------------------------------------------------------------------
// strided passes (y, z)
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_strided(SParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  // y inverse of a solve: work-group 0 takes the stop decision, the tiles
  // start at work-group 1
  const int dec = MODE == ST_INV ? p.decide : 0;
  if (MODE == ST_INV && dec && blockIdx.x == 0) {
    pcg_decide(p.tab.s[p.batch.slot[blockIdx.y]], p.dec);
    return;
  }
  cplx<T>* work = p.work;
  const SolveState* st = nullptr;
  double* part_delta = nullptr;
  if (work == nullptr) {
    const Slot<T> sl = p.tab.s[p.batch.slot[blockIdx.y]];
    if (solve_stopped(sl.st)) return;
    work = sl.work;
    st = sl.st;
    part_delta = sl.part_delta;
  }
  const int B = p.B, lgB = p.lgB, L = p.L, Lin = p.Lin;
  const int pen0 = (blockIdx.x - dec) * B;
  for (int e = tid; e < (Lin << lgB); e += kThreads) {
    const int b = e & (B - 1);
    const int t = e >> lgB;
    const int pen = pen0 + b;
    cplx<T> v = cmk(T(0), T(0));
    if (pen < p.npencils) {
      const int grp = pen / p.per_group;
      const size_t base = (size_t)grp * p.group_stride + (pen - grp * p.per_group);
      v = work[base + (size_t)t * p.elem_stride];
    }
    buf[e] = v;
  }
  for (int e = tid; e < ((L - Lin) << lgB); e += kThreads) buf[(Lin << lgB) + e] = cmk(T(0), T(0));
  __syncthreads();
  if constexpr (MODE == ST_INV) {
    lds_fft<T, true>(buf, L, lgB, p.rp, p.tw);
  } else {
    lds_fft<T, false>(buf, L, lgB, p.rp, p.tw);
  }
  if constexpr (MODE == ST_CONV) {
    const int Lyh = p.Ly / 2 + 1;
    double dacc = 0.0;              // (v, r) by Parseval, as in the two-level passes
    for (int e = tid; e < (L << lgB); e += kThreads) {
      const int b = e & (B - 1);
      const int t = e >> lgB;
      const int pen = pen0 + b;
      if (pen < p.npencils) {
        const int ky = pen / p.Kx;
        const int kx = pen - ky * p.Kx;
        const int kyf = min(ky, p.Ly - ky);
        const int kzf = min(t, p.Lz - t);
        T m = p.table[((size_t)kzf * Lyh + kyf) * p.Kx + kx];
        if (p.k0_from_slot && pen == 0 && t == 0) m = T(st->g0);
        const cplx<T> w = buf[e];
        dacc += double(half_bin_weight(kx, p.Lx)) * double(m) *
                (double(w.x) * double(w.x) + double(w.y) * double(w.y));
        buf[e] = cscale(w, m);
      }
    }
    if (part_delta) {
      const double sd = block_sum(dacc);
      if (tid == 0) part_delta[blockIdx.x] = sd;
    }
    __syncthreads();
    lds_fft<T, true>(buf, L, lgB, p.rp, p.tw);
  }
  for (int e = tid; e < (p.Lout << lgB); e += kThreads) {
    const int b = e & (B - 1);
    const int t = e >> lgB;
    const int pen = pen0 + b;
    if (pen < p.npencils) {
      const int grp = pen / p.per_group;
      const size_t base = (size_t)grp * p.group_stride + (pen - grp * p.per_group);
      work[base + (size_t)t * p.elem_stride] = buf[e];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Work-groups of the generic x passes (also the count of their partials).
template <typename T> static int generic_xpass_groups(const XParams<T>& p) {
  const int npairs = (p.nrows + 1) / 2;
  return (npairs + p.P - 1) / p.P;
}

// Partials of the solve-mode x passes: one per wavefront in the two-level
// passes, one per work-group in the generic ones.
template <typename T> int xpass_parts(const XParams<T>& p) {
  if (fast_length(p.g.Lx)) return fast_xpass_parts(p.g.Lx, p.nrows);
  return generic_xpass_groups(p);
}

template <typename T> void launch_xfwd(int mode, const XParams<T>& p, hipStream_t s) {
  if (mode != XF_GEN_FREE && fast_length(p.g.Lx) && fast_xfwd<T>(mode, p, s)) return;
  const dim3 grid(generic_xpass_groups(p), p.has_slots ? p.batch.n : 1);
  const size_t lds = (size_t)p.P * p.g.Lx * sizeof(cplx<T>);
  if (mode == XF_SOLVE) GPS_LAUNCH((k_xfwd<T, XF_SOLVE>), grid, dim3(kThreads), lds, s, p);
  else if (mode == XF_REAL) GPS_LAUNCH((k_xfwd<T, XF_REAL>), grid, dim3(kThreads), lds, s, p);
  else GPS_LAUNCH((k_xfwd<T, XF_GEN_FREE>), grid, dim3(kThreads), lds, s, p);
}

template <typename T> void launch_xinv(int mode, const XParams<T>& p, hipStream_t s) {
  if (fast_length(p.g.Lx) && fast_xinv<T>(mode, p, s)) return;
  const dim3 grid(generic_xpass_groups(p), p.has_slots ? p.batch.n : 1);
  const size_t lds = (size_t)p.P * p.g.Lx * sizeof(cplx<T>);
  if (mode == XI_SOLVE) GPS_LAUNCH((k_xinv<T, XI_SOLVE>), grid, dim3(kThreads), lds, s, p);
  else GPS_LAUNCH((k_xinv<T, XI_REAL>), grid, dim3(kThreads), lds, s, p);
}

template <typename T> int strided_parts(const SParams<T>& p) {
  if (fast_length(p.L)) return fast_strided_parts<T>(p);
  return (p.npencils + p.B - 1) / p.B;
}

template <typename T> void launch_strided(int mode, const SParams<T>& p, hipStream_t s) {
  if (fast_length(p.L) && fast_strided<T>(mode, p, s)) return;
  const int dec = mode == ST_INV && p.decide ? 1 : 0;   // the decision work-group
  const dim3 grid((p.npencils + p.B - 1) / p.B + dec, p.work ? 1 : p.batch.n);
  const size_t lds = (size_t)p.B * p.L * sizeof(cplx<T>);
  if (mode == ST_FWD) GPS_LAUNCH((k_strided<T, ST_FWD>), grid, dim3(kThreads), lds, s, p);
  else if (mode == ST_INV) GPS_LAUNCH((k_strided<T, ST_INV>), grid, dim3(kThreads), lds, s, p);
  else GPS_LAUNCH((k_strided<T, ST_CONV>), grid, dim3(kThreads), lds, s, p);
}

template int strided_parts<float>(const SParams<float>&);
template int strided_parts<double>(const SParams<double>&);
template int xpass_parts<float>(const XParams<float>&);
template int xpass_parts<double>(const XParams<double>&);
template void launch_xfwd<float>(int, const XParams<float>&, hipStream_t);
template void launch_xfwd<double>(int, const XParams<double>&, hipStream_t);
template void launch_xinv<float>(int, const XParams<float>&, hipStream_t);
template void launch_xinv<double>(int, const XParams<double>&, hipStream_t);
template void launch_strided<float>(int, const SParams<float>&, hipStream_t);
template void launch_strided<double>(int, const SParams<double>&, hipStream_t);

}  // namespace gps
