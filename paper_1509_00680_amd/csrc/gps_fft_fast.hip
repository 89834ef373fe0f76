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
// Pencils per tile of a strided pass: FastTile<T>::B, except for FP32 passes
// of length 320 and 384, which take 8.  Their 16-pencil LDS tile (L x 17
// values, 46-55 KB) fits 2-3 work-groups per CU; the 8-pencil tile fits 5-6,
// which hides more of the latency of the transforms (160^3: z pass 52.5 ->
// 41.5 us, y passes 23.8 / 22.4 -> 21.7 / 21.8 us; 128 x 128 x 192 slab, z
// length 384: 22.3 -> 16.2 us).  At the shorter lengths the 16-pencil tile
// already fits 4 or more, and its 128-byte rows are whole cache lines.
template <typename T> int strided_tile(int, int L) {
  return (L >= 320 && FastTile<T>::B == 16) ? 8 : FastTile<T>::B;
}
// Row pairs per work-group of the x passes: 6, and 10 at length 320 (L1 =
// 20).  Every x-forward work-group re-sums the x-inverse's partials, one per
// work-group, so that head costs the square of the work-group count; at
// 160^3 (12,800 row pairs) 10 pairs take the x forward from 39.1 to 32.2 us
// (8 and 12 pairs: 36.1 us); on the 96^3 and 128 x 128 x 192 grids 6 pairs
// are fastest.
template <int L1> constexpr int xpairs() { return L1 == 20 ? 10 : 6; }

constexpr int round64(int v) { return (v + 63) / 64 * 64; }

template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return cmk(a.x, -a.y); }

// Store of a value that the next kernel reads on other XCDs (the transposes
// around the z pass): non-temporal, so the line does not stay dirty in this
// XCD's L2 until the end-of-kernel write-back.  Large outputs of the y-forward
// and z passes (plain_store: 32 MiB and more, 66 MB at 160^3) are stored
// plainly instead: they then stay in the last-level cache for the next pass
// (160^3: z pass 57.8 -> 52.5 us after a plain y forward; y inverse 25.3 ->
// 22.3 us after a plain z pass).
template <typename T>
__device__ __forceinline__ void store_stream(cplx<T>* dst, cplx<T> v) {
  __builtin_nontemporal_store(v.x, &dst->x);
  __builtin_nontemporal_store(v.y, &dst->y);
}

// ---------------------------------------------------------------------------
// strided passes
// ---------------------------------------------------------------------------
// A work-group transforms NTILE adjacent tiles of B pencils.  Every global load
// of all its tiles is issued first, so the later tiles' loads are in flight
// while the first tile is transformed.  PAD: the pencil holds L/2 data points
// (Hockney zero padding): the forward and z passes read, and the inverse and z
// passes write, only the first L/2 elements, and the zero half is a
// compile-time constant.
template <typename T, int L1, int L2, int MODE, bool PAD, int NTILE, int B, bool PLAIN>
__global__ __launch_bounds__(round64(B * L1))
void k_fstrided(SParams<T> p) {
  constexpr int L = L1 * L2;
  constexpr int PITCH = B + 1;
  constexpr int NT = round64(B * L1);
  __shared__ cplx<T> lds[L * PITCH];
  __shared__ cplx<T> twl[L];
  const int tid = threadIdx.x;
  // y inverse of a solve: work-group 0 only takes the stop decision (it runs
  // beside the transforms instead of after one); the tiles are numbered from
  // work-group 1 on
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
    work = sl.work;
    st = sl.st;
    part_delta = sl.part_delta;
  }
  // twiddles first, then the tile, then the stop flag: all in flight together
  cplx<T> twv[(L + NT - 1) / NT];
#pragma unroll
  for (int i = 0; i < (L + NT - 1) / NT; ++i)
    twv[i] = p.tw[min(tid + i * NT, L - 1)];    // clamped: no branch around the load
  const int b = tid & (B - 1);
  const int q = tid / B;
  // (xcd_tile maps work-group 0 to tile 0, so the shift keeps every XCD's
  // tiles contiguous)
  const int tile0 = (xcd_tile(blockIdx.x, gridDim.x) - dec) * NTILE;
  // 32-bit byte offsets: the longest compile-time length is 384, so every
  // buffer these passes index is below 4 GiB
  constexpr unsigned CB = sizeof(cplx<T>);
  const unsigned es = CB * (unsigned)p.elem_stride;
  // Element e of this thread's pencil sits at base + e * es.  Every element a
  // thread touches has e = q + L1 k or e = q + L2 k (k compile-time), so its
  // offset is qb + k * (L1 es) or qb + k * (L2 es): one per-thread product
  // (es < 2^24 for every compile-time length) and scalar steps.
  const unsigned s1 = (unsigned)L1 * es, s2 = (unsigned)L2 * es;
  int pen[NTILE];
  bool pv[NTILE];
  unsigned base[NTILE], qb[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) {
    pen[t] = (tile0 + t) * B + b;
    pv[t] = pen[t] < p.npencils;
    base[t] = 0;
    if (pv[t]) {
      const unsigned grp = fast_div((unsigned)pen[t], p.div_group);
      base[t] = CB * (grp * (unsigned)p.group_stride + ((unsigned)pen[t] - grp * (unsigned)p.per_group));
    }
    qb[t] = base[t] + __umul24((unsigned)q, es);
  }
  // data extents: PAD bounds the input of the forward and z passes and the
  // output of the inverse and z passes
  const int lin = (PAD && MODE != ST_INV) ? L / 2 : p.Lin;
  const int lout = (PAD && MODE != ST_FWD) ? L / 2 : p.Lout;

  // ---- phase 1: every load of every tile (the stop flag is read after them,
  // so both travel together: a stopped solve wastes the loads, never a round
  // trip) ----
  cplx<T> xin[MODE != ST_INV ? NTILE : 1][L1];
  cplx<T> yin[MODE == ST_INV ? NTILE : 1][L2];
  T gm[MODE == ST_CONV ? NTILE : 1][MODE == ST_CONV ? L2 : 1];
  T gw[NTILE];                                  // z pass: half-spectrum weight of the pencil
#pragma unroll
  for (int t = 0; t < NTILE; ++t) {
    if constexpr (MODE != ST_INV) {
      if (q < L2) {
#pragma unroll
        for (int n1 = 0; n1 < L1; ++n1) {
          // branch-free: a clamped element (base 0 for pencils past the end)
          // is loaded and then selected, so the loads issue back to back
          const int e = L2 * n1 + q;
          if (PAD && n1 >= L1 / 2) {
            xin[t][n1] = cmk(T(0), T(0));
          } else if (PAD) {
            // no select: a lane past the last pencil (offset 0) transforms
            // real data and stores nothing
            xin[t][n1] = at_bytes(work, qb[t] + (unsigned)n1 * s2);
          } else {
            // clamped to element lin - 1 (branch-free)
            const unsigned o = e < lin ? qb[t] + (unsigned)n1 * s2 : base[t] + (unsigned)(lin - 1) * es;
            const cplx<T> v = at_bytes(work, o);
            xin[t][n1] = (pv[t] && e < lin) ? v : cmk(T(0), T(0));
          }
        }
      }
      if constexpr (MODE == ST_CONV) {
        // spectrum multipliers of the z pass: prefetched with the tile
        {
          // branch-free: a lane past the last pencil reads pencil 0's entries,
          // and a thread with q >= L1 (NT is B * L1 rounded up to a wavefront)
          // reads those of q = 0; neither is used
          const int Lyh = p.Ly / 2 + 1;
          const int pc = pv[t] ? pen[t] : 0;
          const int qc = q < L1 ? q : 0;
          const int ky = (int)fast_div((unsigned)pc, p.div_kx);
          const int kx = pc - ky * p.Kx;
          gw[t] = T(half_bin_weight(kx, p.Lx));
          const int kyf = min(ky, p.Ly - ky);
          const unsigned row = (unsigned)sizeof(T) * (unsigned)(kyf * p.Kx + kx);
          const unsigned zs = (unsigned)sizeof(T) * (unsigned)(Lyh * p.Kx);
          // folded index min(kz, L - kz) of kz = qc + L1 k2: two arithmetic
          // progressions in k2 and a select (zs < 2^24)
          const unsigned up = row + __umul24((unsigned)qc, zs);
          const unsigned down = row + __umul24((unsigned)(L - qc), zs);
          const unsigned zstep = (unsigned)L1 * zs;
#pragma unroll
          for (int k2 = 0; k2 < L2; ++k2) {
            const unsigned o = qc <= L / 2 - L1 * k2 ? up + (unsigned)k2 * zstep
                                                      : down - (unsigned)k2 * zstep;
            gm[t][k2] = at_bytes(p.table, o);
          }
        }
      }
    } else {
      if (q < L1) {
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) {
          const int kk = q + L1 * k2;
          if (PAD) {
            // full-length input (kk < L): no select, as above
            yin[t][k2] = at_bytes(work, qb[t] + (unsigned)k2 * s1);
          } else {
            // clamped to element lin - 1 (branch-free, as above)
            const unsigned o = kk < lin ? qb[t] + (unsigned)k2 * s1 : base[t] + (unsigned)(lin - 1) * es;
            const cplx<T> v = at_bytes(work, o);
            yin[t][k2] = (pv[t] && kk < lin) ? v : cmk(T(0), T(0));
          }
        }
      }
    }
  }
  const int flag = st ? stop_flag_issue(st) : 0;
#pragma unroll
  for (int i = 0; i < (L + NT - 1) / NT; ++i)
    if (tid + i * NT < L) twl[tid + i * NT] = twv[i];
  if (stop_flag_set(flag)) return;
  __syncthreads();
  const cplx<T>* tw = twl;

  // ---- phase 2: transform the tiles one after the other ----
  double dacc = 0.0;                            // z pass: this thread's part of (v, r)
#pragma unroll
  for (int t = 0; t < NTILE; ++t) {
    if (t > 0) __syncthreads();                 // previous tile's LDS reads are done
    cplx<T> y[L2];
    if constexpr (MODE != ST_INV) {
      if (q < L2) {
        cplx<T> x[L1];
#pragma unroll
        for (int n1 = 0; n1 < L1; ++n1) x[n1] = xin[t][n1];
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
        reg_fft<T, false, L2>(y);               // y[k2] = X[q + L1 k2]
      }
      if constexpr (MODE == ST_FWD) {
        if (pv[t] && q < L1) {
#pragma unroll
          for (int k2 = 0; k2 < L2; ++k2) {
            const int kk = q + L1 * k2;
            if (kk < lout) {
              if constexpr (PLAIN) at_bytes(work, qb[t] + (unsigned)k2 * s1) = y[k2];
              else store_stream(&at_bytes(work, qb[t] + (unsigned)k2 * s1), y[k2]);
            }
          }
        }
        continue;
      } else {
        if (pv[t] && q < L1) {
          // (v, r) = sum over the full spectrum of m |w^|^2 (Parseval), taken
          // as Re(conj(w^) m w^); this pencil's half-spectrum bin k_x stands for
          // itself and its mirror (weight gw)
          // (products of the bulk type, summed in FP64 like every inner product)
          double ws = 0.0;
#pragma unroll
          for (int k2 = 0; k2 < L2; ++k2) {
            const int kz = q + L1 * k2;
            T m = gm[t][k2];
            if (p.k0_from_slot && pen[t] == 0 && kz == 0) m = T(st->g0);
            const cplx<T> w = y[k2];
            y[k2] = cscale(w, m);
            ws += double(y[k2].x) * double(w.x) + double(y[k2].y) * double(w.y);
          }
          dacc += double(gw[t]) * ws;
        }
        __syncthreads();                        // step-2 reads of lds are done
      }
    } else {
      if (q < L1) {
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) y[k2] = yin[t][k2];
      }
    }
    // inverse transform (ST_CONV second half, ST_INV)
    if (q < L1) {
      reg_fft<T, true, L2>(y);                  // y[n_a] = Z[q][n_a]
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
      reg_fft<T, true, L1>(x);                  // x[n_b] = out[q + L2 n_b]
      if (pv[t]) {
#pragma unroll
        for (int nb = 0; nb < L1; ++nb) {
          const int e = q + L2 * nb;
          const bool out = PAD ? (nb < L1 / 2) : (e < lout);
          if (out) {
            if constexpr (MODE == ST_CONV) {
              if constexpr (PLAIN) at_bytes(work, qb[t] + (unsigned)nb * s2) = x[nb];
              else store_stream(&at_bytes(work, qb[t] + (unsigned)nb * s2), x[nb]);
            }
            else at_bytes(work, qb[t] + (unsigned)nb * s2) = x[nb];
          }
        }
      }
    }
  }
  if constexpr (MODE == ST_CONV) {
    if (part_delta) {                           // one partial per wavefront
      const double sd = wave_sum(dacc);
      if ((tid & 63) == 0) part_delta[blockIdx.x * (NT / 64) + (tid >> 6)] = sd;
    }
  }
}

// ---------------------------------------------------------------------------
// x passes (pairs of real rows packed as one complex row)
// ---------------------------------------------------------------------------
// A work-group transforms 2P consecutive rows.  Row lengths are compile-time
// (PAD: the box holds L/2 points of the padded length L, else L), so every
// loop has a fixed trip count and all global loads of a thread are issued
// before the first one is used.
template <int L1> constexpr int xthreads() { return round64(xpairs<L1>() * L1); }

// Work-group sum for a compile-time block of NT threads: one wavefront needs
// no barrier.
template <int NT>
__device__ __forceinline__ double wg_sum(double v) {
  if constexpr (NT == 64) return wave_sum(v);
  else return block_sum(v);
}

// (row, column) of the element e = tid + i NT of a row-major tile with
// compile-time row length W, advanced in i without a division per element.
template <int W, int NT>
struct RowCol {
  int row, col;
  __device__ __forceinline__ explicit RowCol(int tid) : row(tid / W), col(tid - (tid / W) * W) {}
  __device__ __forceinline__ void next() {
    col += NT % W;
    row += NT / W;
    if (col >= W) {
      col -= W;
      ++row;
    }
  }
};

// Element idx of a buffer with a work-group-uniform base, addressed through a
// 32-bit byte offset (the buffers of the compile-time lengths are < 4 GiB).
#define GPS_AT(ptr, idx) at_bytes((ptr), (unsigned)(idx) * (unsigned)sizeof(*(ptr)))

// Work-buffer offsets of the NR consecutive rows row0, row0 + 1, ... of a
// tile (0 for rows past nrows).  row0 is work-group uniform, so the one division runs on the scalar
// unit and the offsets stay in scalar registers.
template <int NR, typename T>
__device__ __forceinline__ void tile_row_offsets(const XParams<T>& p, int row0, int Kx,
                                                 unsigned* off, bool* ok) {
  int pl = row0 / p.rows_per_plane;
  int rr = row0 - pl * p.rows_per_plane;
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    ok[j] = row0 + j < p.nrows;
    // rows past the end get offset 0, so that unconditional loads stay in bounds
    off[j] = ok[j] ? (unsigned)pl * (unsigned)p.plane_stride + (unsigned)rr * (unsigned)Kx : 0u;
    if (++rr == p.rows_per_plane) {
      rr = 0;
      ++pl;
    }
  }
}

template <typename T, int L1, int L2, int MODE, bool PAD>
__global__ __launch_bounds__(xthreads<L1>())
void k_fxfwd(XParams<T> p) {
  constexpr bool SOLVE = MODE == XF_SOLVE || MODE == XF_SOLVE_REF;
  constexpr bool REF = MODE == XF_SOLVE_REF;     // also s += alpha sigma (refinement)
  constexpr int P = xpairs<L1>();
  constexpr int L = L1 * L2;
  constexpr int PITCH = P + 1;
  constexpr int NT = xthreads<L1>();
  constexpr int Lin = PAD ? L / 2 : L;
  constexpr int Kx = L / 2 + 1;
  constexpr int NIN = 2 * P * Lin;                 // real inputs of the tile
  constexpr int EIN = (NIN + NT - 1) / NT;
  constexpr int KI = (Kx + NT - 1) / NT;           // output bins per thread and row pair
  __shared__ cplx<T> lds[L * PITCH];
  __shared__ cplx<T> twl[L];
  T* ldsr = reinterpret_cast<T*>(lds);
  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int row0 = tile * 2 * P;
  cplx<T>* work = p.work;
  const Slot<T> sl = p.tab.s[p.batch.slot[blockIdx.y]];
  if constexpr (SOLVE) work = sl.work;
  constexpr int ETW = (L + NT - 1) / NT;
  cplx<T> twv[ETW];
#pragma unroll
  for (int i = 0; i < ETW; ++i)
    twv[i] = p.tw[min(tid + i * NT, L - 1)];    // clamped: no branch around the load
  // the head's own loads (state words, (p, Ap) partials) go first, then the
  // operands of the r update and of the transform (r, 1/sqrt(eps), Ap), then
  // those of the phi (and s) update (p, phi), which are used only after the
  // transform: the head waits only for its loads, the transform only for the
  // first group, and the second group arrives while the transform runs.
  // Operands are loaded even at k = 0 (unused there).
  XHead<NT == 64 ? 24 : 8> hd;                     // one (p, Ap) partial per x-inverse group
  if constexpr (SOLVE) xfwd_head_load(sl, p.n_pap_parts, hd);
  // rows are contiguous (row stride Lin, checked by the dispatcher), so
  // element e of the tile is at row0 * Lin + e
  const unsigned eo = (unsigned)row0 * (unsigned)Lin;
  const int nin = min(NIN, (p.nrows - row0) * Lin);     // tile elements that exist
  T rv[EIN], sv[EIN], pv[EIN], av[EIN];
  double fv[EIN];
  double gv[REF ? EIN : 1], cv[REF ? EIN : 1];   // sigma, s
  // Loads are unconditional: elements past the tile's end load its first
  // element (unused).  Without branches around the loads the compiler counts
  // them exactly and waits for each group alone.
#pragma unroll
  for (int i = 0; i < EIN; ++i) {
    const int e = tid + i * NT;
    const bool in = e < nin;
    const unsigned o = eo + (unsigned)(in ? e : 0);
    if constexpr (SOLVE) {
      const T r0 = GPS_AT(sl.r, o), s0 = GPS_AT(sl.isq, o);
      av[i] = GPS_AT(sl.ap, o);
      rv[i] = in ? r0 : T(0);
      sv[i] = in ? s0 : T(0);
    } else {
      const T r0 = T(GPS_AT(p.in_real, o));
      rv[i] = in ? r0 : T(0);
      sv[i] = T(0);
    }
  }
  if constexpr (SOLVE) {
#pragma unroll
    for (int i = 0; i < EIN; ++i) {
      const int e = tid + i * NT;
      const unsigned o = eo + (unsigned)(e < nin ? e : 0);
      pv[i] = GPS_AT(sl.p, o);
      fv[i] = GPS_AT(sl.phi, o);
      if constexpr (REF) {
        gv[i] = GPS_AT(sl.sig64, o);
        cv[i] = GPS_AT(sl.src64, o);
      }
    }
  }
  double alpha = 0.0;
  bool upd = false;
  if constexpr (SOLVE) {
    int k;
    if (!xfwd_head_finish(sl, p.n_pap_parts, hd, &k, &alpha, &upd)) return;
  }
  // phase 2: update, scale, stage the rows in LDS
  double mu = 0.0, rr = 0.0;
  // LDS float index of (row, x): 2 (x PITCH + row / 2) + row % 2 = 2 PITCH x + row
  RowCol<Lin, NT> rc(tid);
#pragma unroll
  for (int i = 0; i < EIN; ++i, rc.next()) {
    const int e = tid + i * NT;
    if (e < NIN) {
      T a = rv[i];
      if constexpr (SOLVE) {
        if (e < nin) {
          const unsigned o = eo + (unsigned)e;
          if (upd) {
            a = a - T(alpha) * av[i];
            GPS_AT(sl.r, o) = a;
          }
          rr += double(a) * double(a);
          a = a * sv[i];
          mu += double(a);
        }
      }
      ldsr[__umul24(2 * PITCH, (unsigned)rc.col) + rc.row] = a;
    }
  }
  if constexpr (PAD) {
#pragma unroll
    for (int i = 0; i < (P * (L - Lin) + NT - 1) / NT; ++i) {
      const int e = tid + i * NT;
      if (e < P * (L - Lin)) lds[(Lin + e / P) * PITCH + (e % P)] = cmk(T(0), T(0));
    }
  }
#pragma unroll
  for (int i = 0; i < ETW; ++i)
    if (tid + i * NT < L) twl[tid + i * NT] = twv[i];
  __syncthreads();
  const int pp = tid % P;
  const int q = tid / P;
  const cplx<T>* tw = twl;
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
  unsigned roff[2 * P];
  bool rok[2 * P];
  tile_row_offsets<2 * P>(p, row0, Kx, roff, rok);
#pragma unroll
  for (int p2 = 0; p2 < P; ++p2) {
#pragma unroll
    for (int i = 0; i < KI; ++i) {
      const int kk = tid + i * NT;
      if (kk < Kx) {
        const cplx<T> zk = lds[kk * PITCH + p2];
        const cplx<T> zm = lds[(kk == 0 ? 0 : L - kk) * PITCH + p2];
        const T half = T(0.5);
        if (rok[2 * p2])
          GPS_AT(work, roff[2 * p2] + kk) = cmk(half * (zk.x + zm.x), half * (zk.y - zm.y));
        if (rok[2 * p2 + 1])
          GPS_AT(work, roff[2 * p2 + 1] + kk) = cmk(half * (zk.y + zm.y), half * (zm.x - zk.x));
      }
    }
  }
  if constexpr (SOLVE) {
    // phi += alpha p (and s += alpha sigma) of the previous iteration, after
    // the transform so that its operands' latency hides behind it
    if (upd) {
#pragma unroll
      for (int i = 0; i < EIN; ++i) {
        const int e = tid + i * NT;
        if (e < nin) {
          const unsigned o = eo + (unsigned)e;
          GPS_AT(sl.phi, o) = fv[i] + alpha * double(pv[i]);
          if constexpr (REF) GPS_AT(sl.src64, o) = cv[i] + alpha * gv[i];
        }
      }
    }
  }
  if constexpr (SOLVE) {                        // one partial per work-group
    const double s2 = wg_sum<NT>(rr);
    if (tid == 0) sl.part_rr[tile] = s2;
    if (p.periodic_mean) {
      const double s = wg_sum<NT>(mu);
      if (tid == 0) sl.part_mu[tile] = s;
    }
  }
}

// MODE XI_SOLVE / XI_SOLVE_PERIODIC / XI_SOLVE_REF: v = u / sqrt(eps) and the
// direction update of the PCG iteration (with the periodic mean term; with the
// refinement's sigma = r / sqrt(eps) + beta sigma); XI_REAL: plain output.
template <typename T, int L1, int L2, int MODE, bool PAD>
__global__ __launch_bounds__(xthreads<L1>())
void k_fxinv(XParams<T> p) {
  constexpr bool SOLVE = MODE != XI_REAL;
  constexpr bool PER = MODE == XI_SOLVE_PERIODIC;
  constexpr bool REF = MODE == XI_SOLVE_REF;
  constexpr int P = xpairs<L1>();
  constexpr int L = L1 * L2;
  constexpr int PITCH = P + 1;
  constexpr int NT = xthreads<L1>();
  constexpr int Lout = PAD ? L / 2 : L;
  constexpr int Kx = L / 2 + 1;
  constexpr int KI = (Kx + NT - 1) / NT;           // input bins per thread and row pair
  constexpr int NOUT = 2 * P * Lout;
  constexpr int EOUT = (NOUT + NT - 1) / NT;
  __shared__ cplx<T> lds[L * PITCH];
  __shared__ cplx<T> twl[L];
  const T* ldsr = reinterpret_cast<const T*>(lds);
  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int row0 = tile * 2 * P;
  cplx<T>* work = p.work;
  const Slot<T> sl = p.tab.s[p.batch.slot[blockIdx.y]];
  if constexpr (SOLVE) work = sl.work;
  // the y-inverse decision of this iteration (plain loads: written by an
  // earlier kernel, first used in the epilogue)
  DirArgs dir{};
  if constexpr (SOLVE) {
    dir.fresh = sl.st->fresh;
    dir.beta = sl.st->beta;
    dir.mu = PER ? sl.st->mu : 0.0;
  }
  constexpr int ETW = (L + NT - 1) / NT;
  cplx<T> twv[ETW];
#pragma unroll
  for (int i = 0; i < ETW; ++i)
    twv[i] = p.tw[min(tid + i * NT, L - 1)];    // clamped: no branch around the load
  unsigned roff[2 * P];
  bool rok[2 * P];
  tile_row_offsets<2 * P>(p, row0, Kx, roff, rok);
  cplx<T> xa[P][KI], xb[P][KI];
#pragma unroll
  for (int p2 = 0; p2 < P; ++p2) {
#pragma unroll
    for (int i = 0; i < KI; ++i) {
      const int kk = tid + i * NT;
      const int kc = kk < Kx ? kk : Kx - 1;        // clamped: branch-free loads
      const cplx<T> va = GPS_AT(work, roff[2 * p2] + kc);
      const cplx<T> vb = GPS_AT(work, roff[2 * p2 + 1] + kc);
      xa[p2][i] = rok[2 * p2] ? va : cmk(T(0), T(0));
      xb[p2][i] = rok[2 * p2 + 1] ? vb : cmk(T(0), T(0));
    }
  }
  // the stop flag right after the rows: the transform waits for both, and the
  // epilogue operands below stay in flight while it runs
  int stop = 0;
  if constexpr (SOLVE) stop = stop_flag_issue(sl.st);
  // epilogue operands are independent of the transform: load them now too
  constexpr int EO = SOLVE ? EOUT : 1;
  T sv[EO], rv[EO], qv[EO], pv[EO], av[EO], mv[PER ? EOUT : 1];
  double gv[REF ? EOUT : 1];                     // sigma
  // rows are contiguous (row stride Lout, checked by the dispatcher)
  const unsigned eo = (unsigned)row0 * (unsigned)Lout;
  const int nout = min(NOUT, (p.nrows - row0) * Lout);  // tile elements that exist
  if constexpr (SOLVE) {
    // unconditional loads (elements past the tile's end load its first
    // element, unused): no branches, so the transform waits for the row loads
    // alone
#pragma unroll
    for (int i = 0; i < EOUT; ++i) {
      const int e = tid + i * NT;
      const unsigned o = eo + (unsigned)(e < nout ? e : 0);
      sv[i] = GPS_AT(sl.isq, o);
      rv[i] = GPS_AT(sl.r, o);
      qv[i] = GPS_AT(sl.qk, o);
      pv[i] = GPS_AT(sl.p, o);
      av[i] = GPS_AT(sl.ap, o);
      if constexpr (PER) mv[i] = GPS_AT(sl.s, o);
      if constexpr (REF) gv[i] = GPS_AT(sl.sig64, o);
    }
    if (stop_flag_set(stop)) return;
  }
#pragma unroll
  for (int p2 = 0; p2 < P; ++p2)
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int kk = tid + i * NT;
    if (kk < Kx) {
      cplx<T> a = xa[p2][i], b = xb[p2][i];
      if (kk == 0 || 2 * kk == L) {    // self-conjugate bins of a real row
        a.y = T(0);
        b.y = T(0);
      }
      lds[kk * PITCH + p2] = cmk(a.x - b.y, a.y + b.x);
      const int km = L - kk;
      if (kk > 0 && km >= Kx) lds[km * PITCH + p2] = cmk(a.x + b.y, b.x - a.y);
    }
  }
#pragma unroll
  for (int i = 0; i < ETW; ++i)
    if (tid + i * NT < L) twl[tid + i * NT] = twv[i];
  __syncthreads();
  const int pp = tid % P;
  const int q = tid / P;
  const cplx<T>* tw = twl;
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
  if constexpr (SOLVE) {
    double acc = 0.0;
    RowCol<Lout, NT> rc(tid);
#pragma unroll
    for (int i = 0; i < EOUT; ++i, rc.next()) {
      const int e = tid + i * NT;
      if (e < nout) {
        const unsigned o = eo + (unsigned)e;
        const T v = ldsr[__umul24(2 * PITCH, (unsigned)rc.col) + rc.row] * sv[i];
        T pn = pv[i], an = av[i];
        if constexpr (REF) {
          const double w = double(rv[i] * sv[i]);   // the preconditioner input of this iteration
          GPS_AT(sl.sig64, o) = dir.fresh ? w : w + dir.beta * gv[i];
        }
        direction_update(v, rv[i], qv[i], PER ? mv[i] : T(0), pn, an, dir);
        GPS_AT(sl.p, o) = pn;
        GPS_AT(sl.ap, o) = an;
        acc += double(pn) * double(an);
      }
    }
    const double s1 = wg_sum<NT>(acc);          // one partial per work-group
    if (tid == 0) sl.part_pap[tile] = s1;
  } else {
    RowCol<Lout, NT> rc(tid);
#pragma unroll
    for (int i = 0; i < EOUT; ++i, rc.next()) {
      const int e = tid + i * NT;
      if (e < nout) GPS_AT(p.out_real, eo + (unsigned)e) = double(ldsr[__umul24(2 * PITCH, (unsigned)rc.col) + rc.row]);
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

static int xpass_pairs(int L) {
  switch (L) {
#define GPS_CASE(LL, A, BB) case LL: return xpairs<A>();
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
    default: return 6;
  }
}

int fast_xpass_groups(int L, int nrows) {
  const int P = xpass_pairs(L);
  return ((nrows + 1) / 2 + P - 1) / P;
}

// Partials of the solve-mode x passes: one per work-group.
int fast_xpass_parts(int L, int nrows) { return fast_xpass_groups(L, nrows); }

// Tiles per work-group of the strided passes.
constexpr int kStridedTiles = 1;

template <typename T> int fast_strided_groups(int npencils, int B) {
  const int W = B * kStridedTiles;
  return (npencils + W - 1) / W;
}

// z pass (solve mode): one partial per wavefront
template <typename T> int fast_strided_parts(const SParams<T>& p) {
  const int B = strided_tile<T>(ST_CONV, p.L);
  switch (p.L) {
#define GPS_CASE(LL, A, BB) \
  case LL: return fast_strided_groups<T>(p.npencils, B) * (round64(B * A) / 64);
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
    default: return 0;
  }
}
template int fast_strided_parts<float>(const SParams<float>&);
template int fast_strided_parts<double>(const SParams<double>&);

template <typename T>
bool fast_strided(int mode, const SParams<T>& p, hipStream_t s) {
  constexpr int NTL = kStridedTiles;
  // PAD when the pencil's data half is L/2: forward reads, z pass reads and
  // writes, inverse writes that half only
  const bool pad = (mode == ST_FWD && 2 * p.Lin == p.L) ||
                   (mode == ST_CONV && 2 * p.Lin == p.L && p.Lout == p.Lin) ||
                   (mode == ST_INV && 2 * p.Lout == p.L && p.Lin == p.L);
  const int dec = mode == ST_INV && p.decide ? 1 : 0;   // the decision work-group
  constexpr int BT = FastTile<T>::B;
  constexpr int BS = 8;                                  // FP32 passes at lengths 320, 384
  const int B = strided_tile<T>(mode, p.L);
  const bool plain = p.plain_store != 0;
  const dim3 grid(fast_strided_groups<T>(p.npencils, B) + dec, p.work ? 1 : p.batch.n);
// k_fstrided<T, L1, L2, mode, pad, NTL, B, plain>
#define GPS_K(A, BB, M, P, BX, PL) k_fstrided<T, A, BB, M, P, NTL, BX, PL>
#define GPS_PASS(A, BB, P)                                                                     \
  if (mode == ST_FWD) {                                                                        \
    if (B != BT) { if (plain) GPS_LAUNCH((GPS_K(A, BB, ST_FWD, P, BS, true)), grid, blk, 0, s, p); \
      else GPS_LAUNCH((GPS_K(A, BB, ST_FWD, P, BS, false)), grid, blk, 0, s, p); }           \
    else if (plain) GPS_LAUNCH((GPS_K(A, BB, ST_FWD, P, BT, true)), grid, blk, 0, s, p);       \
    else GPS_LAUNCH((GPS_K(A, BB, ST_FWD, P, BT, false)), grid, blk, 0, s, p);                 \
  } else if (mode == ST_INV) {                                                                 \
    if (B != BT) GPS_LAUNCH((GPS_K(A, BB, ST_INV, P, BS, false)), grid, blk, 0, s, p);         \
    else GPS_LAUNCH((GPS_K(A, BB, ST_INV, P, BT, false)), grid, blk, 0, s, p);                 \
  } else if (B == BT) {                                                                        \
    if (plain) GPS_LAUNCH((GPS_K(A, BB, ST_CONV, P, BT, true)), grid, blk, 0, s, p);           \
    else GPS_LAUNCH((GPS_K(A, BB, ST_CONV, P, BT, false)), grid, blk, 0, s, p);                \
  } else {                                                                                     \
    if (plain) GPS_LAUNCH((GPS_K(A, BB, ST_CONV, P, BS, true)), grid, blk, 0, s, p);           \
    else GPS_LAUNCH((GPS_K(A, BB, ST_CONV, P, BS, false)), grid, blk, 0, s, p);                \
  }
  switch (p.L) {
#define GPS_CASE(LL, A, BB)                                                                    \
  case LL: {                                                                                   \
    const dim3 blk(round64(B * A));                                                            \
    if (pad) {                                                                                 \
      GPS_PASS(A, BB, true)                                                                    \
    } else {                                                                                   \
      GPS_PASS(A, BB, false)                                                                   \
    }                                                                                          \
    return true;                                                                               \
  }
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
#undef GPS_PASS
#undef GPS_K
    default: return false;
  }
}

// x passes exist for full rows (Lin = L) and for half-padded rows (Lin = L/2).
template <typename T>
bool fast_xfwd(int mode, const XParams<T>& p, hipStream_t s) {
  if (mode != XF_SOLVE && mode != XF_REAL) return false;
  const bool pad = 2 * p.Lin == p.g.Lx;
  if (!pad && p.Lin != p.g.Lx) return false;
  if (p.in_row_stride != p.Lin) return false;        // the kernels assume contiguous rows
  const dim3 grid(fast_xpass_groups(p.g.Lx, p.nrows), p.has_slots ? p.batch.n : 1);
  switch (p.g.Lx) {
#define GPS_CASE(LL, A, BB)                                                                      \
  case LL: {                                                                                     \
    const dim3 blk(xthreads<A>());                                                      \
    if (mode == XF_SOLVE && p.refine) {                                                          \
      if (pad) GPS_LAUNCH((k_fxfwd<T, A, BB, XF_SOLVE_REF, true>), grid, blk, 0, s, p);          \
      else GPS_LAUNCH((k_fxfwd<T, A, BB, XF_SOLVE_REF, false>), grid, blk, 0, s, p);             \
    } else if (mode == XF_SOLVE) {                                                               \
      if (pad) GPS_LAUNCH((k_fxfwd<T, A, BB, XF_SOLVE, true>), grid, blk, 0, s, p);      \
      else GPS_LAUNCH((k_fxfwd<T, A, BB, XF_SOLVE, false>), grid, blk, 0, s, p);         \
    } else {                                                                                     \
      if (pad) GPS_LAUNCH((k_fxfwd<T, A, BB, XF_REAL, true>), grid, blk, 0, s, p);       \
      else GPS_LAUNCH((k_fxfwd<T, A, BB, XF_REAL, false>), grid, blk, 0, s, p);          \
    }                                                                                            \
    return true;                                                                                 \
  }
    GPS_FAST_LENGTHS(GPS_CASE)
#undef GPS_CASE
    default: return false;
  }
}

template <typename T>
bool fast_xinv(int mode, const XParams<T>& p, hipStream_t s) {
  const bool pad = 2 * p.Lout == p.g.Lx;
  if (!pad && p.Lout != p.g.Lx) return false;
  if (p.in_row_stride != p.Lout) return false;       // the kernels assume contiguous rows
  const dim3 grid(fast_xpass_groups(p.g.Lx, p.nrows), p.has_slots ? p.batch.n : 1);
  switch (p.g.Lx) {
#define GPS_CASE(LL, A, BB)                                                                      \
  case LL: {                                                                                     \
    const dim3 blk(xthreads<A>());                                                      \
    if (mode == XI_SOLVE && p.periodic_mean) {                                                   \
      if (pad) GPS_LAUNCH((k_fxinv<T, A, BB, XI_SOLVE_PERIODIC, true>), grid, blk, 0, s, p);     \
      else GPS_LAUNCH((k_fxinv<T, A, BB, XI_SOLVE_PERIODIC, false>), grid, blk, 0, s, p);        \
    } else if (mode == XI_SOLVE && p.refine) {                                                   \
      if (pad) GPS_LAUNCH((k_fxinv<T, A, BB, XI_SOLVE_REF, true>), grid, blk, 0, s, p);          \
      else GPS_LAUNCH((k_fxinv<T, A, BB, XI_SOLVE_REF, false>), grid, blk, 0, s, p);             \
    } else if (mode == XI_SOLVE) {                                                               \
      if (pad) GPS_LAUNCH((k_fxinv<T, A, BB, XI_SOLVE, true>), grid, blk, 0, s, p);              \
      else GPS_LAUNCH((k_fxinv<T, A, BB, XI_SOLVE, false>), grid, blk, 0, s, p);                 \
    } else {                                                                                     \
      if (pad) GPS_LAUNCH((k_fxinv<T, A, BB, XI_REAL, true>), grid, blk, 0, s, p);               \
      else GPS_LAUNCH((k_fxinv<T, A, BB, XI_REAL, false>), grid, blk, 0, s, p);                  \
    }                                                                                            \
    return true;                                                                                 \
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
