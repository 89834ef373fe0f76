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

// Head of the x-forward pass, the first kernel of an iteration: takes the
// iteration number k from the state (and publishes it for the other kernels
// of the iteration); for k >= 1, alpha_{k-1} = delta_{k-1} / (p_{k-1}, A p_{k-1}).
// Returns false (whole work-group) if the solve has stopped or (p, Ap) >= 0
// (loss of definiteness).
template <typename T>
__device__ __forceinline__ bool xfwd_head(const Slot<T>& sl, int n_pap_parts, int* k_out,
                                          double* alpha_out) {
  if (wg_read_flag(&sl.st->done)) return false;
  const int k = wg_read_flag(&sl.st->k_next);
  if (blockIdx.x == 0 && threadIdx.x == 0) sl.st->k = k;
  *k_out = k;
  double alpha = 0.0;
  if (k > 0) {
    const double pap = sum_partials(sl.part_pap, n_pap_parts);
    if (!(pap < 0.0)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        sl.st->status = isfinite(pap) ? GPS_E_BREAKDOWN : GPS_E_NONFINITE;
        sl.st->iters = k - 1;
        sl.st->done = 1;
      }
      return false;
    }
    alpha = sl.hist[(size_t)(k - 1) * 4 + 0] / pap;
    if (blockIdx.x == 0 && threadIdx.x == 0) sl.hist[(size_t)(k - 1) * 4 + 2] = alpha;
  }
  *alpha_out = alpha;
  return true;
}

// Head of the direction kernel, the last kernel of iteration k: stop decision
// on ||r_k||^2 (and, at k = 0, on the input checks of the init kernel), then
// delta_k = (v_k, r_k) > 0.  Returns false (whole work-group) if the solve
// stops here; otherwise advances the iteration counter.
template <typename T>
__device__ __forceinline__ bool direction_head(const Slot<T>& sl, int n_x_parts,
                                               int n_vec_parts, int check_neutral, int* k_out,
                                               double* delta_out) {
  if (wg_read_flag(&sl.st->done)) return false;
  const int k = wg_read_flag(&sl.st->k);
  *k_out = k;
  const double rr = sum_partials(sl.part_rr, n_x_parts);
  const double delta = sum_partials(sl.part_delta[0], n_x_parts);
  double thr2, rsum = 0.0, rabs = 0.0;
  int status = -1;
  if (k == 0) {
    rsum = sum_partials(sl.part_init + 1, n_vec_parts, 4);
    rabs = sum_partials(sl.part_init + 2, n_vec_parts, 4);
    const int err = wg_read_flag(&sl.st->err);
    thr2 = fmax(sl.st->abs_thr * sl.st->abs_thr, sl.st->rel_thr * sl.st->rel_thr * rr);
    if (err & kErrNonFinite) status = GPS_E_NONFINITE;
    else if (err & kErrEpsNonPositive) status = GPS_E_INVALID;
    else if (check_neutral && fabs(rsum) > 1e-10 * rabs) status = GPS_E_INVALID;
  } else {
    thr2 = *reinterpret_cast<const volatile double*>(&sl.st->thr2);
  }
  if (status < 0) {
    if (!isfinite(rr)) status = GPS_E_NONFINITE;
    else if (rr <= thr2) status = GPS_OK;
    else if (k >= sl.maxit) status = GPS_E_NOT_CONVERGED;
    else if (!(delta > 0.0)) status = isfinite(delta) ? GPS_E_BREAKDOWN : GPS_E_NONFINITE;
  }
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
      sl.st->k_next = k + 1;
    }
  }
  *delta_out = delta;
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
