// Internal declarations shared by the HIP translation units of libgps.
// Not part of the public ABI (see include/gps.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace gps {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;

// Threads per work-group for every kernel of the library.
constexpr int kThreads = 256;
// LDS tile of an FFT pass, in complex elements (32 KiB FP32, 63 KiB FP64:
// with the reduction scratch a work-group stays under 64 KiB of LDS).
template <typename T> struct TileCap;
template <> struct TileCap<float> { static constexpr int elems = 4096; static constexpr int max_batch = 16; };
template <> struct TileCap<double> { static constexpr int elems = 4032; static constexpr int max_batch = 8; };

// Elements per thread of the pointwise kernels; a work-group covers
// kThreads * kVec consecutive grid points.
constexpr int kVec = 8;

// Work-groups (and FP64 partials) of a pointwise kernel over n points.
__host__ __device__ inline int vec_groups(long long n) {
  return (int)((n + (long long)kThreads * kVec - 1) / ((long long)kThreads * kVec));
}

// Work-groups of the q kernel (one point per thread); at most kVec *
// vec_groups(n), the size of the part_aux array.
__host__ __device__ inline int qfield_groups(long long n) {
  return (int)((n + kThreads - 1) / kThreads);
}

// Division of a non-negative n < 2^31 by a divisor d >= 1 fixed at launch:
// q = (mulhi(n, m) + n) >> s with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1 (Granlund and Montgomery's round-up
// method; mulhi(n, m) <= n, so the sum fits 32 bits).  Replaces the ~15
// instructions of a runtime integer division in per-thread index math.
struct FastDiv {
  unsigned m;
  int s;
};
inline FastDiv make_fastdiv(unsigned d) {
  int s = 0;
  while ((1ull << s) < d) ++s;
  const unsigned long long m = (((1ull << s) - d) << 32) / d + 1;
  return FastDiv{(unsigned)m, s};
}
__device__ __forceinline__ unsigned fast_div(unsigned n, FastDiv f) {
  return (__umulhi(n, f.m) + n) >> f.s;
}

// Largest grid (points) of gps_polarization_charge_noalloc; its scratch array
// holds this many doubles (32 MiB) per GPU.
constexpr long long kNoAllocMaxPoints = 4194304;

constexpr int kMaxStages = 16;
constexpr int kMaxLen = 1024;        // longest supported FFT length

template <typename T> struct cplx { T x, y; };

// Mixed-radix factorisation of one FFT length (radices 2, 3, 4, 5, 7).
struct RadixPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
};

// Convergence / status words of one solve, resident in device memory.
struct SolveState {
  int done;          // 1 once the solve has stopped (any reason)
  int status;        // gps_status value once done
  int iters;         // iterations completed
  int err;           // input-check flags raised by the init kernel
  int k;             // current iteration (written by the x-forward pass)
  int k_next;        // next iteration (written by the y-inverse decision)
  double rr0;        // ||r_0||^2
  double thr2;       // stop threshold on ||r||^2
  double rr;         // last ||r||^2
  double rho_sum;    // sum rho, sum |rho| and sum rho^2 of the right-hand side
  double rho_abs;
  double rho_sq;
  // per-solve parameters (set by the reset kernel)
  double abs_thr;    // absolute stop threshold on ||r||
  double rel_thr;    // relative stop threshold on ||r|| / ||r_0||
  double g0;         // periodic k = 0 multiplier of the preconditioner
  double delta[2];   // delta_k = (v_k, r_k) at index k & 1 (y-inverse decision)
  double beta;       // beta_k of the current iteration (y-inverse decision)
  double mu;         // mean of r_k / sqrt(eps) (periodic; y-inverse decision)
  int restart;       // set by a refinement: the next iteration applies no update and
                     // starts a new direction (cleared by the y-inverse decision)
  int fresh;         // this iteration starts a direction: p = v (y-inverse decision)
  int rel_from_b;    // warm start: the relative threshold is taken on ||4 pi rho||, not ||r_0||
  // nonlinear outer loop (Algorithm SCPBimproved), decided on the device after
  // each inner solve (k_outer_decide); kept across the reset of the inner state
  int outer_done;    // 1 once the outer loop has stopped (status in outer_status)
  int outer_status;
  double outer_res;  // ||rho_ion,k+1 - rho_ion,k||_2 / ||rho||_2 of the last outer step
};

// Input-check flags (SolveState::err)
constexpr int kErrEpsNonPositive = 1;
constexpr int kErrNonFinite = 2;

// Device-resident pointers of one problem in flight.  T is the bulk type
// (float in mixed precision, double in plain FP64).
template <typename T> struct Slot {
  T *r, *p, *ap;              // PCG vectors (v_k lives only in registers)
  T *isq;                     // 1/sqrt(eps)
  T *qk;                      // q + kappa2 (fixed operator diagonal)
  T *s;                       // sqrt(eps) (periodic mean term; may be null)
  T *ion, *ion_prev;          // ionic charge (nonlinear PB only)
  double *phi;                // solution accumulator (FP64)
  double *sig64, *src64;      // refinement: source of p and of phi (FP64; null when off)
  double *qk64;               // refinement: q + kappa2 in FP64 (null when off)
  double *sq64;               // sqrt(eps) in FP64 (stencil input)
  cplx<T> *work;              // FFT work buffer  nz * Ly * Kx
  double *part_init;          // 4 partial sums per init work-group
  double *part_rr;            // ||r||^2 partials (x-forward work-groups)
  double *part_delta;         // (v, r) partials (z-pass work-groups)
  double *part_pap;           // (p, Ap) partials (x-inverse work-groups)
  double *part_mu;            // sum r/sqrt(eps) partials (periodic; x-forward work-groups)
  double *part_aux;           // q-kernel (1 per 256 points), ionic-update / energy (2 per WG)
  double *hist;               // per-iteration history: delta, beta, alpha, ||r||^2
  SolveState *st;
  int maxit;
  int hist_cap;
};

// Problems per launch.  The slot table travels by value in the kernel
// arguments (constant memory), so a work-group finds its buffers without a
// dependent global load, and a captured graph stays valid across solves.
constexpr int kArgSlots = 8;
template <typename T> struct SlotTable {
  Slot<T> s[kArgSlots];
};

// Problems of one batched launch: blockIdx.y indexes these arrays.  Each
// problem keeps its own iteration counter in its SolveState, so a launch
// (or a replayed graph of launches) needs no per-iteration arguments.
struct Batch {
  int n;
  int slot[kArgSlots];        // index into the slot table
};

// Geometry of one plan, passed by value to kernels.
struct Geom {
  int nx, ny, nz;             // box
  int Lx, Ly, Lz;             // FFT lengths
  int Kx;                     // Lx/2 + 1
  int periodic_x, periodic_y, periodic_z;
  double h;
};

}  // namespace gps
