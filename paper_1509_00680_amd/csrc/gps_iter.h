// Convergence decision at the head of a PCG iteration (shared by the x-pass
// kernels of both FFT families).
#pragma once

#include "gps_device.h"
#include "gps.h"

namespace gps {

// ---------------------------------------------------------------------------
// iteration head: convergence decision at the start of PCG iteration k
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool iteration_head(const Slot<T>& sl, int k, int n_vec_parts, int check_neutral) {
  if (wg_read_flag(&sl.st->done)) return false;
  double rr, thr2 = 0.0, rsum = 0.0, rabs = 0.0;
  int status = -1;
  if (k == 0) {
    rr = sum_partials(sl.part_init + 0, n_vec_parts, 4);
    rsum = sum_partials(sl.part_init + 1, n_vec_parts, 4);
    rabs = sum_partials(sl.part_init + 2, n_vec_parts, 4);
    const int err = wg_read_flag(&sl.st->err);
    thr2 = fmax(sl.abs_thr * sl.abs_thr, sl.rel_thr * sl.rel_thr * rr);
    if (err & kErrNonFinite) status = GPS_E_NONFINITE;
    else if (err & kErrEpsNonPositive) status = GPS_E_INVALID;
    else if (check_neutral && fabs(rsum) > 1e-10 * rabs) status = GPS_E_INVALID;
  } else {
    rr = sum_partials(sl.part_rr, n_vec_parts);
    thr2 = *reinterpret_cast<const volatile double*>(&sl.st->thr2);
  }
  if (status < 0) {
    if (!isfinite(rr)) status = GPS_E_NONFINITE;
    else if (rr <= thr2) status = GPS_OK;
    else if (k >= sl.maxit) status = GPS_E_NOT_CONVERGED;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) {
      sl.st->rr0 = rr;
      sl.st->thr2 = thr2;
      sl.st->rho_sum = rsum;
      sl.st->rho_abs = rabs;
    } else if (k - 1 < sl.hist_cap) {
      sl.hist[(size_t)(k - 1) * 4 + 3] = rr;
    }
    sl.st->iters = k;
    sl.st->rr = rr;
    if (status >= 0) {
      sl.st->status = status;
      sl.st->done = 1;
    }
  }
  return status < 0;
}

}  // namespace gps
