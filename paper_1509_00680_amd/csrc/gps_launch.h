// Host-side launchers of the libgps kernels (internal).
#pragma once

#include <hip/hip_ext.h>

#include "gps_internal.h"
#include "gps_iter.h"

namespace gps {

// ---- timed launches ---------------------------------------------------------

// Events that the next launch made on this host thread binds to its dispatch
// (start and end of the kernel's execution, the timestamps a kernel trace
// reports); cleared by that launch.  Both null: plain launch.
struct LaunchEvents {
  hipEvent_t start;
  hipEvent_t stop;
};
LaunchEvents& launch_events();

#define GPS_LAUNCH(kern, grid, blk, shm, strm, ...)                                     \
  do {                                                                                  \
    ::gps::LaunchEvents& gps_ev_ = ::gps::launch_events();                              \
    if (gps_ev_.start) {                                                                \
      const ::gps::LaunchEvents gps_e_ = gps_ev_;                                       \
      gps_ev_ = ::gps::LaunchEvents{nullptr, nullptr};                                  \
      hipExtLaunchKernelGGL(kern, grid, blk, shm, strm, gps_e_.start, gps_e_.stop, 0,   \
                            __VA_ARGS__);                                               \
    } else {                                                                            \
      hipLaunchKernelGGL(kern, grid, blk, shm, strm, __VA_ARGS__);                      \
    }                                                                                   \
  } while (0)

// ---- FFT passes -----------------------------------------------------------

// Pass along x: pairs of real rows -> one complex FFT of length Lx.
// Row `row` of the input is in[row * in_row_stride + x], x < Lin; the output
// row goes to work[(row / rows_per_plane) * plane_stride + (row % rows_per_plane) * Kx + k].
enum XfwdMode { XF_SOLVE = 0, XF_REAL = 1, XF_GEN_FREE = 2 };
// (the two-level x passes have refinement variants XF_SOLVE_REF / XI_SOLVE_REF,
// chosen by XParams::refine; the generic ones test the slot's buffers)
constexpr int XF_SOLVE_REF = 3;
template <typename T> struct XParams {
  Geom g;
  RadixPlan rp;
  const cplx<T>* tw;        // twiddles of length Lx
  int Lin;                  // loaded row length (rest zero)
  int Lout;                 // stored row length (inverse pass)
  int P, lgP;               // row pairs per work-group (power of two)
  int nrows;                // number of real rows
  int rows_per_plane;
  long long plane_stride;   // complex elements between output planes
  long long in_row_stride;  // real elements between input rows
  // XF_REAL / XF_GEN_FREE / XI_REAL: explicit buffers (single problem)
  const double* in_real;
  double* out_real;
  cplx<T>* work;
  // XF_SOLVE / XI_SOLVE: the problems of the batch
  SlotTable<T> tab;
  int has_slots;
  Batch batch;
  int n_pap_parts;          // (p, Ap) partials written by the x-inverse pass
  int periodic_mean;        // periodic: sum r/sqrt(eps) partials and the mean term
  int refine;               // track the FP64 sources sigma and s (true-residual refinement)
};

// x-inverse modes: the PCG epilogue (plain or with the periodic mean term), or
// plain real output.
enum XinvMode { XI_SOLVE = 0, XI_REAL = 1, XI_SOLVE_PERIODIC = 2 };
constexpr int XI_SOLVE_REF = 3;

template <typename T> void launch_xfwd(int mode, const XParams<T>& p, hipStream_t s);
template <typename T> void launch_xinv(int mode, const XParams<T>& p, hipStream_t s);
// Partial sums written by a solve-mode x pass, whichever family runs (at most
// the number of row pairs).
template <typename T> int xpass_parts(const XParams<T>& p);

// Pass along a strided axis: pencils p of length L with elements at
// base(p) + t * elem_stride, base(p) = (p / per_group) * group_stride + p % per_group.
enum StridedMode { ST_FWD = 0, ST_INV = 1, ST_CONV = 2 };
template <typename T> struct SParams {
  RadixPlan rp;
  const cplx<T>* tw;
  int L, Lin, Lout;
  int B, lgB;
  int npencils;
  int per_group;
  FastDiv div_group;        // per_group and Kx as fast divisors (set by the launchers)
  FastDiv div_kx;
  long long group_stride;
  long long elem_stride;
  // ST_CONV: multiply by a real, even table folded to (Lz/2+1)(Ly/2+1)Kx
  const T* table;
  int Kx, Ly, Lz;
  int k0_from_slot;         // periodic: the k = 0 multiplier is the solve state's g0
  int Lx;                   // ST_CONV with slots: x length (weights of the (v, r) partials)
  int decide;               // ST_INV with slots: work-group 0 takes the stop decision
  int plain_store;          // y forward, z pass over 32 MiB and more: ordinary stores (the output
                            // stays in the last-level cache for the next pass)
  DecideArgs dec;
  cplx<T>* work;            // explicit buffer, or null to use the slots
  SlotTable<T> tab;
  Batch batch;
};
template <typename T> void launch_strided(int mode, const SParams<T>& p, hipStream_t s);
// Partial sums written by a solve-mode z pass, whichever family runs (at most
// the number of pencils plus 64).
template <typename T> int strided_parts(const SParams<T>& p);

// Two-level passes for the common lengths (32 ... 384); false if L has none.
bool fast_length(int L);
int fast_xpass_groups(int L, int nrows);
int fast_xpass_parts(int L, int nrows);
template <typename T> int fast_strided_groups(int npencils, int B);
template <typename T> int fast_strided_parts(const SParams<T>& p);   // z pass (solve mode)
template <typename T> bool fast_strided(int mode, const SParams<T>& p, hipStream_t s);
template <typename T> bool fast_xfwd(int mode, const XParams<T>& p, hipStream_t s);
template <typename T> bool fast_xinv(int mode, const XParams<T>& p, hipStream_t s);

// ---- plan-time tables -------------------------------------------------------
void launch_compress_table(const cplx<double>* full, int Kx, int Ly, int Lz, double scale,
                           double* t64, float* t32, hipStream_t s);
void launch_surface_gen(cplx<double>* buf, int Kx, int Lyh, int Lz, int nx, int ny, double h,
                        double k0_offset, hipStream_t s);
void launch_surface_compress(const cplx<double>* buf, int Kx, int Lyh, int Lz, double scale,
                             double* t64, float* t32, hipStream_t s);
void launch_periodic_table(const Geom& g, int laplacian, double* t64, float* t32, hipStream_t s);
// Gauss-Legendre rule on [-1, 1] (nodes, weights) for the wire kernel's cell averages.
constexpr int kGLPoints = 10;
struct GLRule { double t[kGLPoints], w[kGLPoints]; };
void launch_wire_gen(double* out, const Geom& g, double rw, const GLRule& gl, hipStream_t s);


// ---- per-solve vector kernels -------------------------------------------------
struct IonParams {
  int nspecies;
  double Z[4];
  double c[4];
  double a[4];              // c / c_max (0 for Boltzmann)
  int steric;
  double kT;
  double eta;
  double eps_bulk;
  const double* gamma;      // null: (eps - 1)/(eps_bulk - 1)
  const double* eps;
};

template <typename T> void launch_reset_state(const SlotTable<T>& tab, const Batch& b,
                                              double abs_thr, double rel_thr, int rel_from_b,
                                              hipStream_t s);
template <typename T> void launch_idle_state(const SlotTable<T>& tab, const Batch& b,
                                             hipStream_t s);
template <typename T> void launch_set_g0(const SlotTable<T>& tab, const Batch& b, long long n,
                                         double norm, hipStream_t s);
template <typename T> void launch_init(const SlotTable<T>& tab, const Batch& b, const double* rho,
                                       const double* eps, long long n, int keep_src,
                                       hipStream_t s);
template <typename T> void launch_qfield(const SlotTable<T>& tab, const Batch& b, const Geom& g,
                                         int fd_half, const double* lap_sq, double kappa_coef,
                                         const double* eps, const double* gamma,
                                         double eps_bulk, hipStream_t s);
template <typename T> void launch_qcopy(const SlotTable<T>& tab, const Batch& b, long long n,
                                        const double* q, hipStream_t s);
template <typename T> void launch_ion_update(const SlotTable<T>& tab, const Batch& b, long long n,
                                             const IonParams& ip, int first, hipStream_t s);
// One work-group after the ionic update: the outer residual from the update's
// partials (fixed order), the outer decision, and, when the loop goes on, the
// inner state reset for the next outer step (abs_thr, rel_thr_next); when it
// stops, the inner state stays stopped so the launches already queued return.
template <typename T> void launch_outer_decide(const SlotTable<T>& tab, const Batch& b,
                                               int n_parts, double rho_norm, double tol,
                                               double abs_thr, double rel_thr_next, int last,
                                               hipStream_t s);
template <typename T> void launch_energy(const SlotTable<T>& tab, const Batch& b, const double* rho,
                                         long long n, hipStream_t s);
template <typename T> void launch_zero_ion(const SlotTable<T>& tab, const Batch& b, long long n,
                                           hipStream_t s);
template <typename T> void launch_refine(const SlotTable<T>& tab, const Batch& b, const double* rho,
                                         const double* u, long long n, int final_step,
                                         hipStream_t s);

// Cavity builder and diagnostics (gps_cavity.hip)
void launch_rigid_cavity(const Geom& g, const double* atoms, int natoms, double delta,
                         double eps0, double* eps, double* q, hipStream_t s);
void launch_log_field(long long n, const double* eps, double* lne, hipStream_t s);
// Device address of the no-allocation scratch array (kNoAllocMaxPoints
// doubles) on `device`, which must be the current device; looked up once per
// device with hipGetSymbolAddress.
hipError_t noalloc_scratch(int device, double** out);
void launch_polarization(const Geom& g, int fd_half, const double* rho, const double* eps,
                         const double* lne, const double* phi, double* out, hipStream_t s);
int polarization_groups(const Geom& g);
// Planes per z march of the 2.5D stencils over ntxy column tiles.
int stencil_zlen(long long ntxy, int nz);
// Device state of a solve by Algorithm SC or PSD (gps_solve_sc).
struct ScState {
  int done;          // 1 once the solve has stopped
  int status;        // gps_status (GPS_E_NOT_CONVERGED while running)
  int step;          // steps taken
  int iters;         // iterations reported (SC: steps after the first)
  int method;        // gps_sc_method
  int max_steps;
  int pending;       // 1 while the last update waits for its stop decision
  double eta;        // SC mixing
  double thr_w;      // tol ||4 pi rho / eps||
  double thr_r;      // tol ||4 pi rho||
  double thr_sc;     // tol ||rho||
  double rr0;        // ||4 pi rho||^2
  double rr;         // ||r||^2 after the last step
  double ff;         // ||r/eps||^2 after the last step
  double ff_prev;    // ||r/eps||^2 before the last step
  double alpha;      // step of the last iteration
};
// Stop decision of an SC/PSD step from the update's partials (part, nparts
// pairs); st == nullptr: none.
struct ScDecide {
  const double* part;
  int nparts;
  ScState* st;
};
// SC/PSD operator A v = -4 pi r + eps grad ln eps . grad v and two partials
// per work-group (paper_step: (v, r) and (v, A v); else (A v, r/eps^2) and
// (A v, A v/eps^2)); returns at once when *stop != 0 (stop may be null).  With
// dec.st, one extra work-group takes the stop decision of the previous step's
// update (if one is pending) while the others apply the operator.
void launch_sc_operator(const Geom& g, int fd_half, int paper_step, const double* r,
                        const double* eps, const double* lne, const double* v, double* av,
                        double* part, const int* stop, const ScDecide& dec, hipStream_t s);
// The stop decision alone (the last update of a replayed chunk of steps).
void launch_sc_decide(const ScDecide& dec, hipStream_t s);
// Start of an SC/PSD solve: r = -4 pi rho, f = r/eps, phi = 0, eps_c = eps,
// lne = ln eps, and the state (thresholds; done at once for rho = 0 or
// non-finite input).  part: 2 vec_groups(n) doubles of scratch.
void launch_sc_begin(long long n, const double* rho, const double* eps, double* r, double* f,
                     double* phi, double* eps_c, double* lne, double* part, ScState* st,
                     int method, double eta, double tol, int max_steps, hipStream_t s);
// The update of one SC/PSD step: every work-group takes alpha from the
// operator's n_op partial pairs, then phi += alpha v, r -= alpha A v, f =
// r/eps with the ||r||^2, ||f||^2 partials, and marks the step's stop decision
// pending (taken by the next operator launch or launch_sc_decide).  Returns
// at once once the state says done.
void launch_sc_advance(long long n, const double* eps, double* phi, double* r, const double* v,
                       const double* av, double* f, const double* op_part, int n_op,
                       double* part, ScState* st, hipStream_t s);
// (1/2) h^3 sum rho phi partials (one per work-group, stride 2) into part.
void launch_sc_energy(long long n, const double* rho, const double* phi, double* part,
                      hipStream_t s);

}  // namespace gps
