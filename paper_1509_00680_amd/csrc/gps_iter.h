// Scalar steps of a PCG iteration (Algorithm PCG with the Eq. corr identity),
// spread over the five FFT passes of the preconditioner so that an iteration
// needs no kernel of its own:
//
//   x forward   alpha_{k-1} = delta_{k-1} / (p_{k-1}, A p_{k-1}) (every
//               work-group, from the x-inverse partials); phi += alpha p,
//               r -= alpha Ap; w = r / sqrt(eps); partials of ||r_k||^2 and
//               (periodic) sum w.
//   y forward
//   z pass      partials of delta_k = (v_k, r_k), by Parseval on the spectrum
//               it already holds: (r, v) = (w, G w) = sum_k c(k_x) m(k) |w^(k)|^2
//               with m the Green's multiplier applied and c the weight of a
//               half-spectrum bin (1 for k_x = 0 and Nyquist, else 2).
//   y inverse   one extra work-group: stop decision on ||r_k||^2, delta_k,
//               beta_k.
//   x inverse   v_k; A v_k from the Eq. corr identity; p_k = v_k + beta p,
//               Ap_k = A v_k + beta Ap; partials of (p_k, Ap_k).
//
// Every scalar is a fixed-order FP64 sum of per-work-group partials, so a
// solve's bits do not depend on timing.  Only work-group 0 writes the solve
// state.
#pragma once

#include "gps_device.h"
#include "gps.h"

namespace gps {

// Every head loads what it needs (solve-state words, partial sums) in one
// round, before the kernel issues its bulk operand loads.  Vector loads
// retire in order, so the head then waits only for its own loads, and the
// operands arrive while it reduces and decides.

// Partial sums per thread loaded up front; grids with more partials than
// N * blockDim load the remainder when summing.
template <int N>
struct PartShare {
  double v[N];
};

// Branch-free (a clamped index and a select), so that the loads issue back to
// back and nothing waits for them before their use.  n >= 1.
template <int N>
__device__ __forceinline__ void share_load(PartShare<N>& s, const double* __restrict__ p, int n) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int i = threadIdx.x + j * blockDim.x;
    const double v = p[min(i, n - 1)];
    s.v[j] = i < n ? v : 0.0;
  }
}

// Work-group sum of the n partials (fixed order: every work-group of every
// launch gets the same bits).
template <int N>
__device__ __forceinline__ double share_sum(const PartShare<N>& s, const double* __restrict__ p,
                                            int n) {
  static_assert(N % 4 == 0, "share size");
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
  for (int j = 0; j < N; j += 4) {
    a0 += s.v[j];
    a1 += s.v[j + 1];
    a2 += s.v[j + 2];
    a3 += s.v[j + 3];
  }
  const int step = blockDim.x;
  int i = threadIdx.x + N * step;
  for (; i + 3 * step < n; i += 4 * step) {
    const double b0 = p[i], b1 = p[i + step], b2 = p[i + 2 * step], b3 = p[i + 3 * step];
    a0 += b0;
    a1 += b1;
    a2 += b2;
    a3 += b3;
  }
  for (; i < n; i += step) a0 += p[i];
  return block_sum((a0 + a1) + (a2 + a3));
}

// ---- x-forward pass: the first kernel of iteration k ------------------------
// N: (p, Ap) partials per thread held in registers (one partial per x-inverse
// work-group; more are summed from memory).
template <int N = 8>
struct XHead {
  int done, k, restart;
  double dprev0, dprev1;
  PartShare<N> pap;
};

// State words are loaded by every thread (one request per wavefront) with
// plain loads, which wait only where used; thread 0's copy is broadcast, so
// every work-group acts on the same value.
template <typename T, int N>
__device__ __forceinline__ void xfwd_head_load(const Slot<T>& sl, int n_pap_parts, XHead<N>& h) {
  const SolveState* v = sl.st;
  h.done = v->done;
  h.k = v->k_next;
  h.restart = v->restart;
  h.dprev0 = v->delta[0];
  h.dprev1 = v->delta[1];
  share_load(h.pap, sl.part_pap, n_pap_parts);
}

// Takes the iteration number k (and publishes it for the other kernels of the
// iteration); for k >= 1, alpha_{k-1} = delta_{k-1} / (p_{k-1}, A p_{k-1}),
// unless a refinement has just replaced phi and r (then there is no update).
// *upd_out: whether the update of iteration k-1 is applied.  Returns false
// (whole work-group) if the solve has stopped or (p, Ap) >= 0 (loss of
// definiteness).
template <typename T, int N>
__device__ __forceinline__ bool xfwd_head_finish(const Slot<T>& sl, int n_pap_parts,
                                                 const XHead<N>& h, int* k_out,
                                                 double* alpha_out, bool* upd_out) {
  // thread 0's state words, broadcast once: every wavefront of the work-group
  // acts on the same values (work-group 0 may set done during the launch)
  struct Words {
    int done, k, restart;
    double dprev0, dprev1;
  };
  __shared__ Words wb;
  if (threadIdx.x == 0) wb = Words{h.done, h.k, h.restart, h.dprev0, h.dprev1};
  __syncthreads();
  const Words w = wb;
  __syncthreads();
  if (w.done) return false;
  const int k = w.k;
  if (blockIdx.x == 0 && threadIdx.x == 0) sl.st->k = k;
  *k_out = k;
  double alpha = 0.0;
  const bool upd = k > 0 && !w.restart;
  *upd_out = upd;
  if (upd) {
    const double pap = share_sum(h.pap, sl.part_pap, n_pap_parts);
    if (!(pap < 0.0)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        sl.st->status = isfinite(pap) ? GPS_E_BREAKDOWN : GPS_E_NONFINITE;
        sl.st->iters = k - 1;
        sl.st->done = 1;
      }
      return false;
    }
    const double dprev = ((k - 1) & 1) ? w.dprev1 : w.dprev0;
    alpha = dprev / pap;
    if (blockIdx.x == 0 && threadIdx.x == 0) sl.hist[(size_t)(k - 1) * 4 + 2] = alpha;
  }
  *alpha_out = alpha;
  return true;
}

// ---- y-inverse pass, decision work-group: the stop decision of iteration k --
struct DecideArgs {
  int n_rr;            // ||r||^2 and sum w partials (x-forward work-groups)
  int n_delta;         // delta partials (z-pass work-groups)
  int n_init;          // init-kernel work-groups (4 partials each)
  int check_neutral;   // free / surface boundaries: the net charge must vanish
  int periodic;
  double npts;         // grid points (the mean term divides by it)
};

// Stop decision on ||r_k||^2 (and, at k = 0, on the input checks of the init
// kernel); else delta_k = (v_k, r_k) > 0, beta_k = delta_k / delta_{k-1}.
// Writes the solve state (done and status, or delta_k, beta_k, the mean term
// and the next iteration number) for the x-inverse pass.  Run by one
// work-group of the y-inverse launch, beside the transforms; nothing if the
// solve has already stopped.
template <typename T>
__device__ void pcg_decide(const Slot<T>& sl, const DecideArgs& a) {
  SolveState* st = sl.st;
  if (st->done) return;
  PartShare<8> srr, sdl, smu;
  share_load(srr, sl.part_rr, a.n_rr);
  share_load(sdl, sl.part_delta, a.n_delta);
  if (a.periodic) share_load(smu, sl.part_mu, a.n_rr);
  const int k = st->k;
  const double rr = share_sum(srr, sl.part_rr, a.n_rr);
  const double delta = share_sum(sdl, sl.part_delta, a.n_delta);
  const double mu = a.periodic ? share_sum(smu, sl.part_mu, a.n_rr) : 0.0;
  double thr2, rsum = 0.0, rabs = 0.0;
  int status = -1;
  double rr0 = rr;
  if (k == 0) {
    rsum = sum_partials(sl.part_init + 1, a.n_init, 4);
    rabs = sum_partials(sl.part_init + 2, a.n_init, 4);
    // warm start: relative to ||4 pi rho|| (the init kernel's ||r||^2 of phi = 0)
    if (st->rel_from_b) rr0 = sum_partials(sl.part_init + 0, a.n_init, 4);
    const int err = st->err;
    thr2 = fmax(st->abs_thr * st->abs_thr, st->rel_thr * st->rel_thr * rr0);
    if (err & kErrNonFinite) status = GPS_E_NONFINITE;
    else if (err & kErrEpsNonPositive) status = GPS_E_INVALID;
    else if (a.check_neutral && fabs(rsum) > 1e-10 * rabs) status = GPS_E_INVALID;
  } else {
    thr2 = st->thr2;
  }
  if (status < 0) {
    if (!isfinite(rr)) status = GPS_E_NONFINITE;
    else if (rr <= thr2) status = GPS_OK;
    else if (k >= sl.maxit) status = GPS_E_NOT_CONVERGED;
    else if (!(delta > 0.0)) status = isfinite(delta) ? GPS_E_BREAKDOWN : GPS_E_NONFINITE;
  }
  // a new direction at k = 0 and after a refinement
  const int fresh = (k == 0 || st->restart) ? 1 : 0;
  const double beta = fresh ? 0.0 : delta / st->delta[(k - 1) & 1];
  __syncthreads();                       // every thread has read restart
  if (threadIdx.x == 0) {
    if (k == 0) {
      st->rr0 = rr0;
      st->thr2 = thr2;
      st->rho_sum = rsum;
      st->rho_abs = rabs;
    } else {
      sl.hist[(size_t)(k - 1) * 4 + 3] = rr;
    }
    st->iters = k;
    st->rr = rr;
    if (status >= 0) {
      st->status = status;
      st->done = 1;
    } else {
      st->delta[k & 1] = delta;
      st->beta = beta;
      st->fresh = fresh;
      st->restart = 0;
      st->mu = mu / a.npts;
      sl.hist[(size_t)k * 4 + 0] = delta;
      sl.hist[(size_t)k * 4 + 1] = beta;
      st->k_next = k + 1;
    }
  }
}

// Weight of half-spectrum bin kx in a sum over the full spectrum of a real
// field of length Lx along x.
__device__ __forceinline__ int half_bin_weight(int kx, int Lx) {
  return (kx == 0 || 2 * kx == Lx) ? 1 : 2;
}

// ---- x-inverse epilogue: the direction update of iteration k ----------------
// A v = -(q + kappa2) v - 4 pi (r - sqrt(eps) mean(r / sqrt(eps))) [periodic]
// p = v + beta p, Ap = A v + beta Ap (beta = 0 at k = 0).
struct DirArgs {
  int fresh;           // p = v (first iteration, or the first after a refinement)
  double beta;
  double mu;           // mean of r / sqrt(eps) (periodic), else 0
};

template <typename T>
__device__ __forceinline__ void direction_update(T v, T r, T q, T s, T& p, T& ap,
                                                 const DirArgs& d) {
  const T fpi = T(kFourPi);
  const T av = -q * v - fpi * (r - s * T(d.mu));
  if (d.fresh) {
    p = v;
    ap = av;
  } else {
    const T tb = T(d.beta);
    p = v + tb * p;
    ap = av + tb * ap;
  }
}

// x-forward prologue at grid point o (generic passes): apply the update of
// iteration k-1 (phi += alpha p, r -= alpha Ap, and with refinement
// s += alpha sigma), accumulate ||r_k||^2 and return the preconditioner input
// r / sqrt(eps).
template <typename T>
__device__ __forceinline__ T solve_prologue(const Slot<T>& sl, size_t o, bool upd, double alpha,
                                            double& rr) {
  T r = sl.r[o];
  if (upd) {
    const T pv = sl.p[o];
    const T av = sl.ap[o];
    sl.phi[o] += alpha * double(pv);
    r = r - T(alpha) * av;
    sl.r[o] = r;
    if (sl.src64) sl.src64[o] += alpha * sl.sig64[o];
  }
  rr += double(r) * double(r);
  return r * sl.isq[o];
}

// x-inverse epilogue at grid point o (generic passes): v = u / sqrt(eps),
// the direction update, and (p, Ap).
template <typename T>
__device__ __forceinline__ void solve_epilogue(const Slot<T>& sl, size_t o, T u,
                                               const DirArgs& d, bool periodic, double& pap) {
  const T v = u * sl.isq[o];
  T p = sl.p[o], ap = sl.ap[o];
  const T r = sl.r[o];
  if (sl.sig64) {                        // refinement: sigma = r / sqrt(eps) + beta sigma
    const double w = double(r * sl.isq[o]);
    sl.sig64[o] = d.fresh ? w : w + d.beta * sl.sig64[o];
  }
  direction_update(v, r, sl.qk[o], periodic ? sl.s[o] : T(0), p, ap, d);
  sl.p[o] = p;
  sl.ap[o] = ap;
  pap += double(p) * double(ap);
}

}  // namespace gps
