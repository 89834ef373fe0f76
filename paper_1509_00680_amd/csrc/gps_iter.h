// Scalar steps of a PCG iteration, evaluated redundantly (and identically) by
// every work-group of the kernel that needs them, from the FP64 partial sums
// the previous kernel wrote.  Only work-group 0 writes the solve state.
//
// Iteration k runs:  x-forward pass (applies the update of iteration k-1),
// y, z, y-inverse passes, x-inverse pass (v_k, partials of (v_k, r_k) and
// ||r_k||^2), direction kernel (stop decision, beta_k, p_k, Ap_k, partials of
// (p_k, Ap_k)).
#pragma once

#include "gps_device.h"
#include "gps.h"

namespace gps {

// Every head loads what it needs (solve-state words, partial sums) in one
// round, before the kernel issues its bulk operand loads.  Vector loads
// retire in order, so the head then waits only for its own loads, and the
// operands arrive while it reduces and decides.

// Partial sums per thread loaded up front; grids with more partials than
// kHeadShare * blockDim load the remainder when summing.
constexpr int kHeadShare = 8;

struct PartShare {
  double v[kHeadShare];
};

// Branch-free (a clamped index and a select), so that the loads issue back to
// back and nothing waits for them before their use.  n >= 1.
__device__ __forceinline__ void share_load(PartShare& s, const double* __restrict__ p, int n) {
#pragma unroll
  for (int j = 0; j < kHeadShare; ++j) {
    const int i = threadIdx.x + j * blockDim.x;
    const double v = p[min(i, n - 1)];
    s.v[j] = i < n ? v : 0.0;
  }
}

// Work-group sum of the n partials (fixed order: every work-group of every
// launch gets the same bits).
__device__ __forceinline__ double share_sum(const PartShare& s, const double* __restrict__ p,
                                            int n) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
  for (int j = 0; j < kHeadShare; j += 4) {
    a0 += s.v[j];
    a1 += s.v[j + 1];
    a2 += s.v[j + 2];
    a3 += s.v[j + 3];
  }
  for (int i = threadIdx.x + kHeadShare * blockDim.x; i < n; i += blockDim.x) a0 += p[i];
  return block_sum((a0 + a1) + (a2 + a3));
}

// Work-group broadcast of thread 0's value (loaded earlier by thread 0).
template <typename V>
__device__ __forceinline__ V wg_bcast(V w) {
  __shared__ V f;
  if (threadIdx.x == 0) f = w;
  __syncthreads();
  const V r = f;
  __syncthreads();
  return r;
}

// ---- x-forward pass: the first kernel of iteration k ------------------------
struct XHead {
  int done, k;
  double dprev0, dprev1;
  PartShare pap;
};

// State words are loaded by every thread (one request per wavefront) with
// plain loads, which wait only where used; thread 0's copy is broadcast, so a
// work-group acts on one value even when the direction kernel's work-group 0
// writes a word during the same launch.
template <typename T>
__device__ __forceinline__ void xfwd_head_load(const Slot<T>& sl, int n_pap_parts, XHead& h) {
  const SolveState* v = sl.st;
  h.done = v->done;
  h.k = v->k_next;
  h.dprev0 = v->delta[0];
  h.dprev1 = v->delta[1];
  share_load(h.pap, sl.part_pap, n_pap_parts);
}

// Takes the iteration number k (and publishes it for the other kernels of the
// iteration); for k >= 1, alpha_{k-1} = delta_{k-1} / (p_{k-1}, A p_{k-1}).
// Returns false (whole work-group) if the solve has stopped or (p, Ap) >= 0
// (loss of definiteness).
template <typename T>
__device__ __forceinline__ bool xfwd_head_finish(const Slot<T>& sl, int n_pap_parts,
                                                 const XHead& h, int* k_out,
                                                 double* alpha_out) {
  if (wg_bcast(h.done)) return false;
  const int k = wg_bcast(h.k);
  if (blockIdx.x == 0 && threadIdx.x == 0) sl.st->k = k;
  *k_out = k;
  double alpha = 0.0;
  if (k > 0) {
    const double pap = share_sum(h.pap, sl.part_pap, n_pap_parts);
    if (!(pap < 0.0)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        sl.st->status = isfinite(pap) ? GPS_E_BREAKDOWN : GPS_E_NONFINITE;
        sl.st->iters = k - 1;
        sl.st->done = 1;
      }
      return false;
    }
    const double dprev = wg_bcast(((k - 1) & 1) ? h.dprev1 : h.dprev0);
    alpha = dprev / pap;
    if (blockIdx.x == 0 && threadIdx.x == 0) sl.hist[(size_t)(k - 1) * 4 + 2] = alpha;
  }
  *alpha_out = alpha;
  return true;
}

// ---- direction kernel: the last kernel of iteration k -----------------------
struct DHead {
  int done, k, err;
  double thr2, dprev0, dprev1, abs_thr, rel_thr;
  PartShare rr, delta, mu;
};

template <typename T>
__device__ __forceinline__ void direction_head_load(const Slot<T>& sl, int n_x_parts,
                                                    int periodic, DHead& h) {
  const SolveState* v = sl.st;
  h.done = v->done;
  h.k = v->k;
  h.err = v->err;
  h.thr2 = v->thr2;
  h.dprev0 = v->delta[0];
  h.dprev1 = v->delta[1];
  h.abs_thr = v->abs_thr;
  h.rel_thr = v->rel_thr;
  share_load(h.rr, sl.part_rr, n_x_parts);
  share_load(h.delta, sl.part_delta[0], n_x_parts);
  if (periodic) share_load(h.mu, sl.part_mu, n_x_parts);
  else h.mu = PartShare{};
}

// Stop decision on ||r_k||^2 (and, at k = 0, on the input checks of the init
// kernel), then delta_k = (v_k, r_k) > 0 and beta_k = delta_k / delta_{k-1}.
// Returns false (whole work-group) if the solve stops here; otherwise
// advances the iteration counter.
template <typename T>
__device__ __forceinline__ bool direction_head_finish(const Slot<T>& sl, const DHead& h,
                                                      int n_x_parts, int n_vec_parts,
                                                      int check_neutral, int periodic,
                                                      int* k_out, double* delta_out,
                                                      double* beta_out, double* mu_out) {
  if (wg_bcast(h.done)) return false;
  const int k = wg_bcast(h.k);
  *k_out = k;
  const double rr = share_sum(h.rr, sl.part_rr, n_x_parts);
  const double delta = share_sum(h.delta, sl.part_delta[0], n_x_parts);
  *mu_out = periodic ? share_sum(h.mu, sl.part_mu, n_x_parts) : 0.0;
  double thr2, rsum = 0.0, rabs = 0.0;
  int status = -1;
  if (k == 0) {
    // once per solve: the init kernel's partials (a second round)
    rsum = sum_partials(sl.part_init + 1, n_vec_parts, 4);
    rabs = sum_partials(sl.part_init + 2, n_vec_parts, 4);
    const int err = wg_bcast(h.err);
    const double at = wg_bcast(h.abs_thr), rt = wg_bcast(h.rel_thr);
    thr2 = fmax(at * at, rt * rt * rr);
    if (err & kErrNonFinite) status = GPS_E_NONFINITE;
    else if (err & kErrEpsNonPositive) status = GPS_E_INVALID;
    else if (check_neutral && fabs(rsum) > 1e-10 * rabs) status = GPS_E_INVALID;
  } else {
    thr2 = wg_bcast(h.thr2);
  }
  if (status < 0) {
    if (!isfinite(rr)) status = GPS_E_NONFINITE;
    else if (rr <= thr2) status = GPS_OK;
    else if (k >= sl.maxit) status = GPS_E_NOT_CONVERGED;
    else if (!(delta > 0.0)) status = isfinite(delta) ? GPS_E_BREAKDOWN : GPS_E_NONFINITE;
  }
  double beta = 0.0;
  if (k > 0) beta = delta / wg_bcast(((k - 1) & 1) ? h.dprev1 : h.dprev0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) {
      sl.st->rr0 = rr;
      sl.st->thr2 = thr2;
      sl.st->rho_sum = rsum;
      sl.st->rho_abs = rabs;
    } else {
      sl.hist[(size_t)(k - 1) * 4 + 3] = rr;
    }
    sl.st->iters = k;
    sl.st->rr = rr;
    if (status >= 0) {
      sl.st->status = status;
      sl.st->done = 1;
    } else {
      sl.st->delta[k & 1] = delta;
      sl.hist[(size_t)k * 4 + 0] = delta;
      sl.hist[(size_t)k * 4 + 1] = beta;
      sl.st->k_next = k + 1;
    }
  }
  *delta_out = delta;
  *beta_out = beta;
  return status < 0;
}

// x-forward prologue at grid point o: apply the update of iteration k-1
// (phi += alpha p, r -= alpha Ap) and return the preconditioner input
// r / sqrt(eps).
template <typename T>
__device__ __forceinline__ T solve_prologue(const Slot<T>& sl, size_t o, bool upd, double alpha) {
  T r = sl.r[o];
  if (upd) {
    const T pv = sl.p[o];
    const T av = sl.ap[o];
    sl.phi[o] += alpha * double(pv);
    r = r - T(alpha) * av;
    sl.r[o] = r;
  }
  return r * sl.isq[o];
}

// x-inverse epilogue at grid point o: v = u / sqrt(eps); accumulate (v, r)
// and ||r||^2.
template <typename T>
__device__ __forceinline__ void solve_epilogue(const Slot<T>& sl, size_t o, T u, double& vr,
                                               double& rr) {
  const T v = u * sl.isq[o];
  const T r = sl.r[o];
  sl.v[o] = v;
  vr += double(v) * double(r);
  rr += double(r) * double(r);
}

}  // namespace gps
