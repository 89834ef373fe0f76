// Plan, solve drivers and the C ABI of libgps (include/gps.h).
//
// A plan owns, for one grid and boundary condition: the FFT factorisations
// and twiddles of the three axes, the Green's-function spectrum (FP64 and
// FP32 copies, computed on the device at plan time) and, per precision, the
// buffers of one problem in flight.  A solve enqueues the PCG iterations on
// the plan's stream; alpha, beta and the stop decision stay on the device,
// and the host polls the state after a predicted number of iterations.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "gps.h"
#include "gps_internal.h"
#include "gps_launch.h"
#include "gps_batch.h"

using namespace gps;

gps::LaunchEvents& gps::launch_events() {
  static thread_local LaunchEvents ev{nullptr, nullptr};
  return ev;
}

namespace {

// Serializes stream capture against plan creation and destruction across
// host threads (allocation, frees and stream teardown must not overlap another
// thread's capture).
std::mutex g_plan_mu;

struct TimedLaunch {
  int k;
  hipEvent_t start, stop;
};

struct DevError {
  hipError_t e;
};

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw DevError{e};
}

struct NoMem {};

// Capacities of the per-wavefront partial-sum arrays of the solve passes:
// x passes at most one partial per row pair (+1), z pass at most one per
// pencil (+64).
struct PartCaps {
  int x, z;
};
inline PartCaps part_caps(const Geom& g) {
  return PartCaps{(g.ny * g.nz + 1) / 2 + 1, g.Ly * g.Kx + 64};
}
// A launch configuration whose partials would not fit is a library defect;
// it is reported as a device error rather than run.
inline void check_parts(int count, int cap) {
  if (count < 1 || count > cap) throw DevError{hipErrorInvalidConfiguration};
}

template <typename P>
void dalloc(P** p, size_t bytes, size_t* total) {
  *p = nullptr;
  if (bytes == 0) return;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    throw NoMem{};
  }
  *total += bytes;
}

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

bool factorize(int n, RadixPlan* rp) {
  rp->n = n;
  rp->nstages = 0;
  int m = n;
  auto push = [&](int r) {
    if (rp->nstages >= kMaxStages) return false;
    rp->radix[rp->nstages++] = r;
    return true;
  };
  while (m % 4 == 0) { if (!push(4)) return false; m /= 4; }
  if (m % 2 == 0) { if (!push(2)) return false; m /= 2; }
  for (int r : {3, 5, 7}) {
    while (m % r == 0) { if (!push(r)) return false; m /= r; }
  }
  return m == 1 && n <= kMaxLen && n >= 1;
}

int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Per-precision buffers of the problems in flight on a plan: slot 0 for the
// single-solve calls, slots 0..nslots-1 when the plan serves a batch.
template <typename T> struct Res {
  bool ready = false;
  size_t bytes = 0;          // device bytes of this precision's buffers
  SlotTable<T> tab{};        // passed by value to every kernel
  int nslots = 1;            // slots with buffers
  Slot<T>& slot(int i = 0) { return tab.s[i]; }
  SolveState* h_state = nullptr;   // pinned
  double* h_parts = nullptr;       // pinned, >= 4 * groups
  int hist_cap = 0;
  double* lap64 = nullptr;         // periodic spectral Laplacian of sqrt(eps)
  cplx<double>* work64q = nullptr; // FP64 work for the spectral q (mixed + periodic)
  double* u64 = nullptr;           // refinement: G s (FP64)
  bool have_src = false;           // src64 holds the source of the last solve's iterate
  cplx<double>* work64r = nullptr; // refinement: FP64 FFT work buffer
  // graphs of 4, 2 and 1 times `chunk` and of 4, 2 and 1 PCG iterations,
  // longest first (kernel arguments are replay-invariant: the iteration
  // counter lives in the solve state)
  static constexpr int kGraphs = 6;
  hipGraphExec_t graphs[kGraphs] = {};
  int graph_iters[kGraphs] = {};
  int graph_neutral = -1, graph_timing = -1, graph_chunk = 0, graph_refine = -1;
  // batch mode: the same graph lengths over all nslots slots (grid.y = nslots)
  hipGraphExec_t bgraphs[kGraphs] = {};
  int bgraph_iters[kGraphs] = {};
  int bgraph_neutral = -1, bgraph_chunk = 0, bgraph_n = 0;
  SolveState* h_states = nullptr;  // pinned, one per slot
};

template <typename T>
void drop_graphs(Res<T>& R) {
  for (hipGraphExec_t& g : R.graphs) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  for (hipGraphExec_t& g : R.bgraphs) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  R.bgraph_n = 0;
}

}  // namespace


struct gps_plan {
  int device = 0;
  // kernel timing (gps_plan_set_timing)
  int timing_kind = GPS_K_NONE;
  double timing_ms = 0.0;
  long long timing_launches = 0;
  double timing_bytes = 0.0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<TimedLaunch> ev_pending;
  size_t ev_used = 0;
  hipStream_t cap_stream = nullptr;   // side stream used only to capture graphs
  Geom g{};
  int bc = 0;
  gps_options opt{};
  RadixPlan rp[3]{};
  double* tw64[3]{};
  float* tw32[3]{};
  double* green64 = nullptr;
  float* green32 = nullptr;
  double* lap64t = nullptr;     // spectral Laplacian table (periodic)
  double* pol_lne = nullptr;    // ln eps scratch of gps_polarization_charge (n doubles)
  size_t pol_bytes = 0;
  // Algorithm SC / PSD (gps_solve_sc): FP64 fields, partials, device state and
  // captured iteration graphs of 8, 4, 2 and 1 steps
  struct ScRes {
    double *r = nullptr, *v = nullptr, *av = nullptr, *f = nullptr, *lne = nullptr;
    double *eps = nullptr, *phi = nullptr, *part_op = nullptr, *part = nullptr;
    ScState* st = nullptr;
    ScState* h_st = nullptr;      // pinned
    double* h_part = nullptr;     // pinned, 2 vec_groups(n)
    size_t bytes = 0;
    hipGraphExec_t graphs[4] = {};
    int graph_iters[4] = {8, 4, 2, 1};
    int graph_key = -1;           // paper_step + 2 (fd_order/2) + 64 (mixed)
  } sc;
  float* lap32t = nullptr;
  Res<float> r32;
  Res<double> r64;
  size_t bytes = 0;
  gps_info info{};
  std::vector<double> hist;
  long long npts() const { return (long long)g.nx * g.ny * g.nz; }
  hipStream_t stream() const { return reinterpret_cast<hipStream_t>(opt.stream); }
  template <typename T> Res<T>& res();
  template <typename T> const T* green() const;
  template <typename T> const T* lap() const;
  template <typename T> const cplx<T>* tw(int axis) const;
};
template <> Res<float>& gps_plan::res<float>() { return r32; }
template <> Res<double>& gps_plan::res<double>() { return r64; }
template <> const float* gps_plan::green<float>() const { return green32; }
template <> const double* gps_plan::green<double>() const { return green64; }
template <> const float* gps_plan::lap<float>() const { return lap32t; }
template <> const double* gps_plan::lap<double>() const { return lap64t; }
template <> const cplx<float>* gps_plan::tw<float>(int a) const {
  return reinterpret_cast<const cplx<float>*>(tw32[a]);
}
template <> const cplx<double>* gps_plan::tw<double>(int a) const {
  return reinterpret_cast<const cplx<double>*>(tw64[a]);
}

namespace {

// ---------------------------------------------------------------------------
// pass parameter builders
// ---------------------------------------------------------------------------
template <typename T>
XParams<T> xparams(const gps_plan* pl, int nrows, int rows_per_plane, int Lin, int Lout,
                   long long plane_stride, long long in_row_stride) {
  XParams<T> p{};
  p.g = pl->g;
  p.rp = pl->rp[0];
  p.tw = pl->tw<T>(0);
  p.Lin = Lin;
  p.Lout = Lout;
  const int npairs = (nrows + 1) / 2;
  const int cap = std::max(1, TileCap<T>::elems / pl->g.Lx);
  const int want = std::max(1, npairs / 1024);
  p.P = pow2_floor(std::min(cap, want));
  p.lgP = ilog2(p.P);
  p.nrows = nrows;
  p.rows_per_plane = rows_per_plane;
  p.plane_stride = plane_stride;
  p.in_row_stride = in_row_stride;
  return p;
}

template <typename T>
SParams<T> sparams(const gps_plan* pl, int axis, int L, int Lin, int Lout, int npencils,
                   int per_group, long long group_stride, long long elem_stride) {
  SParams<T> p{};
  p.rp = pl->rp[axis];
  p.tw = pl->tw<T>(axis);
  p.L = L;
  p.Lin = Lin;
  p.Lout = Lout;
  const int cap = std::max(1, TileCap<T>::elems / L);
  p.B = pow2_floor(std::min(TileCap<T>::max_batch, cap));
  p.lgB = ilog2(p.B);
  p.npencils = npencils;
  p.per_group = per_group;
  p.div_group = make_fastdiv((unsigned)per_group);
  p.div_kx = make_fastdiv((unsigned)pl->g.Kx);
  p.group_stride = group_stride;
  p.elem_stride = elem_stride;
  p.Kx = pl->g.Kx;
  p.Ly = pl->g.Ly;
  p.Lz = pl->g.Lz;
  // y-forward and z passes over 32 MiB and more of data store plainly (the
  // output stays in the last-level cache for the next pass)
  p.plain_store = axis >= 1 && (long long)Lout * npencils * (long long)sizeof(cplx<T>) >= (32ll << 20);
  return p;
}

// ---------------------------------------------------------------------------
// plan-time Green's-function spectrum (FP64 on the device)
// ---------------------------------------------------------------------------
// Gauss-Legendre nodes and weights on [-1, 1] (Newton's method on the
// Legendre recurrence), for the wire kernel's cell averages.
GLRule gauss_legendre() {
  GLRule r{};
  const int n = kGLPoints;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double pn = 0.0, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      pn = p1;
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    r.t[i] = x;
    r.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return r;
}

void build_green(gps_plan* pl) {
  const Geom& g = pl->g;
  hipStream_t s = pl->cap_stream;
  const size_t ntab = (size_t)(g.Lz / 2 + 1) * (g.Ly / 2 + 1) * g.Kx;
  dalloc(&pl->green64, ntab * sizeof(double), &pl->bytes);
  dalloc(&pl->green32, ntab * sizeof(float), &pl->bytes);
  const double norm = 1.0 / ((double)g.Lx * g.Ly * g.Lz);
  if (pl->bc == GPS_BC_FREE) {
    // K(m) on the full padded grid -> 3D FFT (FP64) -> fold and scale by h^3/N
    const size_t nfull = (size_t)g.Lz * g.Ly * g.Kx;
    size_t tmp_bytes = 0;
    cplx<double>* full = nullptr;
    dalloc(&full, nfull * sizeof(cplx<double>), &tmp_bytes);
    XParams<double> xp = xparams<double>(pl, g.Ly * g.Lz, g.Ly, g.Lx, g.Lx,
                                         (long long)g.Ly * g.Kx, g.Lx);
    xp.work = full;
    launch_xfwd<double>(XF_GEN_FREE, xp, s);
    SParams<double> yp = sparams<double>(pl, 1, g.Ly, g.Ly, g.Ly, g.Lz * g.Kx, g.Kx,
                                         (long long)g.Ly * g.Kx, g.Kx);
    yp.work = full;
    launch_strided<double>(ST_FWD, yp, s);
    SParams<double> zp = sparams<double>(pl, 2, g.Lz, g.Lz, g.Lz / 2 + 1, g.Ly * g.Kx,
                                         g.Ly * g.Kx, 0, (long long)g.Ly * g.Kx);
    zp.work = full;
    launch_strided<double>(ST_FWD, zp, s);
    launch_compress_table(full, g.Kx, g.Ly, g.Lz, g.h * g.h * g.h * norm, pl->green64,
                          pl->green32, s);
    ck(hipGetLastError());
    ck(hipStreamSynchronize(s));
    dfree(full);
  } else if (pl->bc == GPS_BC_WIRE) {
    // per z mode, the cell-averaged in-plane kernel on the (2ny, 2nx) padded
    // plane -> 2D FFT (FP64) -> fold and scale by h^2/N
    const size_t nfull = (size_t)g.Lz * g.Ly * g.Kx;
    size_t tmp_bytes = 0;
    cplx<double>* full = nullptr;
    double* kt = nullptr;
    dalloc(&full, nfull * sizeof(cplx<double>), &tmp_bytes);
    dalloc(&kt, (size_t)g.Lz * g.Ly * g.Lx * sizeof(double), &tmp_bytes);
    const double rw = 2.0 * g.h * std::sqrt((double)g.nx * g.nx + (double)g.ny * g.ny);
    launch_wire_gen(kt, g, rw, gauss_legendre(), s);
    XParams<double> xp = xparams<double>(pl, g.Ly * g.Lz, g.Ly, g.Lx, g.Lx,
                                         (long long)g.Ly * g.Kx, g.Lx);
    xp.in_real = kt;
    xp.work = full;
    launch_xfwd<double>(XF_REAL, xp, s);
    SParams<double> yp = sparams<double>(pl, 1, g.Ly, g.Ly, g.Ly, g.Lz * g.Kx, g.Kx,
                                         (long long)g.Ly * g.Kx, g.Kx);
    yp.work = full;
    launch_strided<double>(ST_FWD, yp, s);
    launch_compress_table(full, g.Kx, g.Ly, g.Lz, g.h * g.h * norm, pl->green64, pl->green32, s);
    ck(hipGetLastError());
    ck(hipStreamSynchronize(s));
    dfree(full);
    dfree(kt);
  } else if (pl->bc == GPS_BC_SURFACE) {
    const int Lyh = g.Ly / 2 + 1;
    const size_t nc = (size_t)g.Kx * Lyh;
    size_t tmp_bytes = 0;
    cplx<double>* buf = nullptr;
    dalloc(&buf, nc * g.Lz * sizeof(cplx<double>), &tmp_bytes);
    // k_par = 0 kernel shifted by 2 pi Lz h (positive definite tent)
    launch_surface_gen(buf, g.Kx, Lyh, g.Lz, g.nx, g.ny, g.h, 2.0 * kPi * g.Lz * g.h, s);
    SParams<double> zp = sparams<double>(pl, 2, g.Lz, g.Lz, g.Lz / 2 + 1, (int)nc, (int)nc, 0,
                                         (long long)nc);
    zp.work = buf;
    launch_strided<double>(ST_FWD, zp, s);
    launch_surface_compress(buf, g.Kx, Lyh, g.Lz, g.h * norm, pl->green64, pl->green32, s);
    ck(hipGetLastError());
    ck(hipStreamSynchronize(s));
    dfree(buf);
  } else {
    launch_periodic_table(g, 0, pl->green64, pl->green32, s);
    dalloc(&pl->lap64t, ntab * sizeof(double), &pl->bytes);
    dalloc(&pl->lap32t, ntab * sizeof(float), &pl->bytes);
    launch_periodic_table(g, 1, pl->lap64t, pl->lap32t, s);
    ck(hipGetLastError());
    ck(hipStreamSynchronize(s));
  }
}

// ---------------------------------------------------------------------------
// per-precision solve resources
// ---------------------------------------------------------------------------
// The buffers of one problem in flight (PCG vectors, fields, FFT work buffer,
// partial sums, state, solution); history and optional buffers separately.
template <typename T>
void alloc_slot(gps_plan* pl, Slot<T>& s, size_t* bytes) {
  const long long n = pl->npts();
  const int nvg = vec_groups(n);
  const Geom& g = pl->g;
  const int nxg = part_caps(g).x;
  const int nzg = part_caps(g).z;
  const size_t nb = (size_t)n * sizeof(T);
  dalloc(&s.r, nb, bytes);
  dalloc(&s.p, nb, bytes);
  dalloc(&s.ap, nb, bytes);
  dalloc(&s.isq, nb, bytes);
  dalloc(&s.qk, nb, bytes);
  if (pl->bc == GPS_BC_PERIODIC) dalloc(&s.s, nb, bytes);
  dalloc(&s.sq64, (size_t)n * sizeof(double), bytes);
  dalloc(&s.work, (size_t)g.nz * g.Ly * g.Kx * sizeof(cplx<T>), bytes);
  dalloc(&s.part_init, (size_t)4 * nvg * sizeof(double), bytes);
  dalloc(&s.part_rr, (size_t)nxg * sizeof(double), bytes);
  dalloc(&s.part_delta, (size_t)nzg * sizeof(double), bytes);
  dalloc(&s.part_pap, (size_t)nxg * sizeof(double), bytes);
  dalloc(&s.part_mu, (size_t)nxg * sizeof(double), bytes);
  dalloc(&s.part_aux, (size_t)kVec * nvg * sizeof(double), bytes);
  dalloc(&s.st, sizeof(SolveState), bytes);
  dalloc(&s.phi, (size_t)n * sizeof(double), bytes);
}

template <typename T>
void free_slot(Slot<T>& s) {
  dfree(s.r); dfree(s.p); dfree(s.ap); dfree(s.isq); dfree(s.qk); dfree(s.s);
  dfree(s.ion); dfree(s.sq64); dfree(s.work); dfree(s.part_init); dfree(s.part_rr);
  dfree(s.part_delta); dfree(s.part_pap); dfree(s.part_mu); dfree(s.part_aux); dfree(s.hist);
  dfree(s.st); dfree(s.phi);
  dfree(s.sig64); dfree(s.src64); dfree(s.qk64);
}

template <typename T>
void ensure_res(gps_plan* pl, bool need_ion, bool need_refine = false) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  Res<T>& R = pl->res<T>();
  const long long n = pl->npts();
  const int nvg = vec_groups(n);
  const Geom& g = pl->g;
  if (!R.ready) {
    R.slot() = Slot<T>{};
    alloc_slot<T>(pl, R.slot(), &R.bytes);
    if (pl->bc == GPS_BC_PERIODIC) {
      dalloc(&R.lap64, (size_t)n * sizeof(double), &R.bytes);
      if (sizeof(T) != sizeof(double))
        dalloc(&R.work64q, (size_t)g.nz * g.Ly * g.Kx * sizeof(cplx<double>), &R.bytes);
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&R.h_state), sizeof(SolveState)) != hipSuccess)
      throw NoMem{};
    if (hipHostMalloc(reinterpret_cast<void**>(&R.h_parts), (size_t)4 * nvg * sizeof(double)) !=
        hipSuccess)
      throw NoMem{};
    R.ready = true;
  }
  if (R.hist_cap < pl->opt.maxit + 1) {
    for (int i = 0; i < R.nslots; ++i) {
      if (R.slot(i).hist) R.bytes -= (size_t)4 * R.hist_cap * sizeof(double);
      dfree(R.slot(i).hist);
      dalloc(&R.slot(i).hist, (size_t)4 * (pl->opt.maxit + 1) * sizeof(double), &R.bytes);
    }
    R.hist_cap = pl->opt.maxit + 1;
  }
  bool changed = false;
  if (need_ion && !R.slot().ion) {
    dalloc(&R.slot().ion, (size_t)n * sizeof(T), &R.bytes);
    changed = true;
  }
  if (need_refine && !R.slot().sig64) {
    Slot<T>& s = R.slot();
    const size_t nd = (size_t)n * sizeof(double);
    dalloc(&s.sig64, nd, &R.bytes);
    dalloc(&s.src64, nd, &R.bytes);
    dalloc(&s.qk64, nd, &R.bytes);
    dalloc(&R.u64, nd, &R.bytes);
    dalloc(&R.work64r, (size_t)g.nz * g.Ly * g.Kx * sizeof(cplx<double>), &R.bytes);
    changed = true;
  }
  // the table is captured by value in graphs: rebuild them when it changes
  if (changed || R.slot().hist_cap != R.hist_cap || R.slot().maxit != pl->opt.maxit)
    drop_graphs(R);
  for (int i = 0; i < R.nslots; ++i) {
    R.slot(i).hist_cap = R.hist_cap;
    R.slot(i).maxit = pl->opt.maxit;
  }
}

template <typename T>
void free_res(gps_plan* pl) {
  Res<T>& R = pl->res<T>();
  drop_graphs(R);
  for (int i = 0; i < R.nslots; ++i) free_slot(R.slot(i));
  dfree(R.lap64); dfree(R.work64q); dfree(R.u64); dfree(R.work64r);
  if (R.h_state) (void)hipHostFree(R.h_state);
  if (R.h_parts) (void)hipHostFree(R.h_parts);
  if (R.h_states) (void)hipHostFree(R.h_states);
  R = Res<T>{};
}

void free_sc(gps_plan* pl) {
  gps_plan::ScRes& S = pl->sc;
  for (hipGraphExec_t& g : S.graphs) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  dfree(S.r); dfree(S.v); dfree(S.av); dfree(S.f); dfree(S.lne); dfree(S.eps); dfree(S.phi);
  dfree(S.part_op); dfree(S.part); dfree(S.st);
  if (S.h_st) (void)hipHostFree(S.h_st);
  if (S.h_part) (void)hipHostFree(S.h_part);
  S = gps_plan::ScRes{};
}

template <typename T>
SolveState read_state(gps_plan* pl) {
  Res<T>& R = pl->res<T>();
  ck(hipMemcpyAsync(R.h_state, R.slot().st, sizeof(SolveState), hipMemcpyDeviceToHost,
                    pl->stream()));
  ck(hipStreamSynchronize(pl->stream()));
  return *R.h_state;
}

// Host sum, in index order, of `count` partials spaced by `stride`.
template <typename T>
double read_sum(gps_plan* pl, const double* dparts, int groups, int stride, int comp) {
  Res<T>& R = pl->res<T>();
  ck(hipMemcpyAsync(R.h_parts, dparts, (size_t)groups * stride * sizeof(double),
                    hipMemcpyDeviceToHost, pl->stream()));
  ck(hipStreamSynchronize(pl->stream()));
  double s = 0.0;
  for (int i = 0; i < groups; ++i) s += R.h_parts[(size_t)i * stride + comp];
  return s;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
hipEvent_t next_event(gps_plan* pl) {
  if (pl->ev_used == pl->ev_pool.size()) {
    hipEvent_t e;
    ck(hipEventCreate(&e));
    pl->ev_pool.push_back(e);
  }
  return pl->ev_pool[pl->ev_used++];
}

// Binds two events to the next launch on stream s: the events take the
// kernel's own start and end timestamps (not the time the stream spent
// reaching it).  Only eager launches are timed.
struct TimerScope {
  gps_plan* pl;
  bool on;
  TimedLaunch tl{};
  TimerScope(gps_plan* p, hipStream_t, int kind, int k) : pl(p), on(p->timing_kind == kind) {
    if (on) {
      tl.k = k;
      tl.start = next_event(pl);
      tl.stop = next_event(pl);
      launch_events() = LaunchEvents{tl.start, tl.stop};
    }
  }
  ~TimerScope() {
    if (on) {
      launch_events() = LaunchEvents{nullptr, nullptr};
      pl->ev_pending.push_back(tl);
    }
  }
};

// After a host sync: add the timed launches of iterations k_base + t.k that
// did work (k < iters_done).
void collect_timing(gps_plan* pl, const std::vector<TimedLaunch>& ev, int k_base,
                    int iters_done) {
  for (const TimedLaunch& t : ev) {
    if (k_base + t.k < iters_done) {
      float ms = 0.f;
      ck(hipEventElapsedTime(&ms, t.start, t.stop));
      pl->timing_ms += ms;
      pl->timing_launches += 1;
    }
  }
}

// Algorithmic bytes of one launch of pass `kind` (inputs read once, outputs
// written once), bulk element size s.
double pass_bytes(const gps_plan* pl, int kind, size_t s) {
  const Geom& g = pl->g;
  const double n = (double)pl->npts();
  const double c = 2.0 * s;
  const double rows = (double)g.ny * g.nz;
  const double wbox = (double)g.nz * g.Ly * g.Kx;   // complex elements of the work buffer
  const double tab = (double)(g.Lz / 2 + 1) * (g.Ly / 2 + 1) * g.Kx;
  const int periodic = pl->bc == GPS_BC_PERIODIC;
  switch (kind) {
    case GPS_K_XFWD: return (5.0 * s + 16.0) * n + rows * g.Kx * c;   // with the fused update
    case GPS_K_YFWD: return (double)g.nz * g.Kx * g.ny * c + wbox * c;
    case GPS_K_ZCONV: return 2.0 * wbox * c + tab * s;
    case GPS_K_YINV: return wbox * c + (double)g.nz * g.Kx * g.ny * c;
    case GPS_K_XINV: return rows * g.Kx * c + (7.0 + periodic) * n * s;   // with the direction update
    default: return 0.0;
  }
}

// ---------------------------------------------------------------------------
// one PCG iteration for the problems of a batch (all of one plan)
// ---------------------------------------------------------------------------
template <typename T>
void enqueue_iteration(gps_plan* pl, const SlotTable<T>& tab, const Batch& b, int check_neutral,
                       hipStream_t s, int k0, int refine) {
  const Geom& g = pl->g;
  const long long n = pl->npts();
  const int periodic = pl->bc == GPS_BC_PERIODIC;
  XParams<T> xp = xparams<T>(pl, g.ny * g.nz, g.ny, g.nx, g.nx, (long long)g.Ly * g.Kx, g.nx);
  xp.tab = tab;
  xp.has_slots = 1;
  xp.batch = b;
  xp.n_pap_parts = xpass_parts(xp);
  xp.refine = refine;
  check_parts(xp.n_pap_parts, part_caps(g).x);
  xp.periodic_mean = periodic;
  { TimerScope t(pl, s, GPS_K_XFWD, k0); launch_xfwd<T>(XF_SOLVE, xp, s); }
  SParams<T> yf = sparams<T>(pl, 1, g.Ly, g.ny, g.Ly, g.nz * g.Kx, g.Kx, (long long)g.Ly * g.Kx,
                             g.Kx);
  yf.tab = tab;
  yf.batch = b;
  { TimerScope t(pl, s, GPS_K_YFWD, k0); launch_strided<T>(ST_FWD, yf, s); }
  SParams<T> zc = sparams<T>(pl, 2, g.Lz, g.nz, g.nz, g.Ly * g.Kx, g.Ly * g.Kx, 0,
                             (long long)g.Ly * g.Kx);
  zc.tab = tab;
  zc.batch = b;
  zc.table = pl->green<T>();
  zc.k0_from_slot = periodic;
  zc.Lx = g.Lx;
  { TimerScope t(pl, s, GPS_K_ZCONV, k0); launch_strided<T>(ST_CONV, zc, s); }
  SParams<T> yi = sparams<T>(pl, 1, g.Ly, g.Ly, g.ny, g.nz * g.Kx, g.Kx, (long long)g.Ly * g.Kx,
                             g.Kx);
  yi.tab = tab;
  yi.batch = b;
  yi.decide = 1;
  yi.dec.n_rr = xp.n_pap_parts;
  yi.dec.n_delta = strided_parts(zc);
  check_parts(yi.dec.n_delta, part_caps(g).z);
  yi.dec.n_init = vec_groups(n);
  yi.dec.check_neutral = check_neutral;
  yi.dec.periodic = periodic;
  yi.dec.npts = double(n);
  { TimerScope t(pl, s, GPS_K_YINV, k0); launch_strided<T>(ST_INV, yi, s); }
  { TimerScope t(pl, s, GPS_K_XINV, k0); launch_xinv<T>(XI_SOLVE, xp, s); }
}

// out = (convolution with the spectrum `table`)(in), all in FP64 with the FP64
// FFT passes on an explicit work buffer.
void apply64(gps_plan* pl, const double* in, double* out, cplx<double>* work,
             const double* table) {
  const Geom& g = pl->g;
  hipStream_t s = pl->stream();
  XParams<double> xp = xparams<double>(pl, g.ny * g.nz, g.ny, g.nx, g.nx,
                                       (long long)g.Ly * g.Kx, g.nx);
  xp.in_real = in;
  xp.out_real = out;
  xp.work = work;
  launch_xfwd<double>(XF_REAL, xp, s);
  SParams<double> yf = sparams<double>(pl, 1, g.Ly, g.ny, g.Ly, g.nz * g.Kx, g.Kx,
                                       (long long)g.Ly * g.Kx, g.Kx);
  yf.work = work;
  launch_strided<double>(ST_FWD, yf, s);
  SParams<double> zc = sparams<double>(pl, 2, g.Lz, g.nz, g.nz, g.Ly * g.Kx, g.Ly * g.Kx, 0,
                                       (long long)g.Ly * g.Kx);
  zc.work = work;
  zc.table = table;
  launch_strided<double>(ST_CONV, zc, s);
  SParams<double> yi = sparams<double>(pl, 1, g.Ly, g.Ly, g.ny, g.nz * g.Kx, g.Kx,
                                       (long long)g.Ly * g.Kx, g.Kx);
  yi.work = work;
  launch_strided<double>(ST_INV, yi, s);
  launch_xinv<double>(XI_REAL, xp, s);
}

// Spectral Laplacian of sqrt(eps) (periodic q) with the FP64 FFT passes.
template <typename T>
void spectral_laplacian(gps_plan* pl, int slot = 0) {
  Res<T>& R = pl->res<T>();
  cplx<double>* work =
      R.work64q ? R.work64q : reinterpret_cast<cplx<double>*>(R.slot(slot).work);
  apply64(pl, R.slot(slot).sq64, R.lap64, work, pl->lap64t);
}

// One true-residual refinement (final: only phi from the source s).
template <typename T>
void refine_step(gps_plan* pl, const double* rho, bool final_step) {
  Res<T>& R = pl->res<T>();
  apply64(pl, R.slot().src64, R.u64, R.work64r, pl->green64);
  Batch b{};
  b.n = 1;
  launch_refine<T>(R.tab, b, rho, R.u64, pl->npts(), final_step ? 1 : 0, pl->stream());
  ck(hipGetLastError());
}

// u = G f with the bulk-precision FFT passes (no sqrt(eps) scaling).
template <typename T>
void vacuum_apply(gps_plan* pl, const double* f, double* u) {
  ensure_res<T>(pl, false);
  Res<T>& R = pl->res<T>();
  const Geom& g = pl->g;
  hipStream_t s = pl->stream();
  cplx<T>* work = R.slot().work;
  XParams<T> xp = xparams<T>(pl, g.ny * g.nz, g.ny, g.nx, g.nx, (long long)g.Ly * g.Kx, g.nx);
  xp.in_real = f;
  xp.out_real = u;
  xp.work = work;
  launch_xfwd<T>(XF_REAL, xp, s);
  SParams<T> yf = sparams<T>(pl, 1, g.Ly, g.ny, g.Ly, g.nz * g.Kx, g.Kx, (long long)g.Ly * g.Kx,
                             g.Kx);
  yf.work = work;
  launch_strided<T>(ST_FWD, yf, s);
  SParams<T> zc = sparams<T>(pl, 2, g.Lz, g.nz, g.nz, g.Ly * g.Kx, g.Ly * g.Kx, 0,
                             (long long)g.Ly * g.Kx);
  zc.work = work;
  zc.table = pl->green<T>();
  launch_strided<T>(ST_CONV, zc, s);
  SParams<T> yi = sparams<T>(pl, 1, g.Ly, g.Ly, g.ny, g.nz * g.Kx, g.Kx, (long long)g.Ly * g.Kx,
                             g.Kx);
  yi.work = work;
  launch_strided<T>(ST_INV, yi, s);
  launch_xinv<T>(XI_REAL, xp, s);
  ck(hipGetLastError());
  ck(hipStreamSynchronize(s));
}

// Capture `chunk` PCG iterations as one graph (rebuilt when the variant
// changes: neutrality check, timed pass).
template <typename T>
void build_graph(gps_plan* pl, int check_neutral, int chunk, int refine) {
  Res<T>& R = pl->res<T>();
  if (R.graphs[0] && R.graph_neutral == check_neutral &&
      R.graph_timing == pl->timing_kind && R.graph_chunk == chunk && R.graph_refine == refine)
    return;
  drop_graphs(R);
  if (!pl->cap_stream) ck(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
  Batch b{};
  b.n = 1;
  b.slot[0] = 0;
  pl->ev_pending.clear();
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto capture = [&](int iters, hipGraphExec_t* out) {
    ck(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < iters; ++j)
      enqueue_iteration<T>(pl, R.tab, b, check_neutral, pl->cap_stream, j, refine);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(pl->cap_stream, &graph);
    if (e != hipSuccess) throw DevError{e};
    const hipError_t e2 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) throw DevError{e2};
  };
  const int sizes[Res<T>::kGraphs] = {4 * chunk, 2 * chunk, chunk, 4, 2, 1};
  for (int i = 0; i < Res<T>::kGraphs; ++i) {
    R.graph_iters[i] = sizes[i];
    capture(sizes[i], &R.graphs[i]);
  }
  R.graph_neutral = check_neutral;
  R.graph_timing = pl->timing_kind;
  R.graph_chunk = chunk;
  R.graph_refine = refine;
}

// Run PCG iterations until the device-side state says done.  Between host
// polls the host enqueues n iterations, n predicted from the recent residual
// decay, as replays of graphs of 4, 2, 1 chunks and 4, 2, 1 iterations, so
// that a solve runs few iterations past its stop decision (those launches
// exit early, but each still loads its operands) with few polls (each leaves
// the GPU idle for about a third of an iteration at 160^3).  first_n > 0 is
// the caller's guess of the iterations needed (the nonlinear outer loop
// passes the previous inner solve's count), else the first batch is two
// chunks.
template <typename T>
SolveState run_pcg(gps_plan* pl, int check_neutral, const double* track_rho = nullptr,
                   int first_n = 0) {
  Res<T>& R = pl->res<T>();
  const int chunk = pl->opt.check_every;
  // track_rho (the right-hand side): the x passes keep the FP64 source s of
  // the iterate, phi is recomputed from it on exit, and with refine_every = m
  // the residual is recomputed every m iterations (batches end there)
  const int track = track_rho != nullptr;
  const int m = track ? pl->opt.refine_every : 0;
  int next_ref = m;
  // Timing needs readable events around single launches; events recorded
  // inside a captured graph cannot be read back, so timed solves launch
  // the same kernels directly on the stream.
  const bool timing = pl->timing_kind != GPS_K_NONE;
  if (!timing) build_graph<T>(pl, check_neutral, chunk, track);
  Batch b{};
  b.n = 1;
  b.slot[0] = 0;
  int k = 0;              // iterations enqueued
  int n = first_n > 0 ? std::min(first_n, 8 * chunk) : 2 * chunk;   // before the next poll
  double prev_rr = -1.0;
  int prev_it = 0;
  SolveState st{};
  for (;;) {
    if (m > 0) n = std::min(n, next_ref - k);
    if (timing) {
      pl->ev_pending.clear();
      pl->ev_used = 0;
      for (int j = 0; j < n; ++j)
        enqueue_iteration<T>(pl, R.tab, b, check_neutral, pl->stream(), j, track);
      ck(hipGetLastError());
    } else {
      // greedy over the graph lengths, longest first: few graph launches
      int left = n;
      for (int i = 0; i < Res<T>::kGraphs; ++i)
        for (; left >= R.graph_iters[i]; left -= R.graph_iters[i])
          ck(hipGraphLaunch(R.graphs[i], pl->stream()));
    }
    const int k_base = k;
    k += n;
    st = read_state<T>(pl);
    if (timing) {
      // launches that did work: up to the stop decision; none when the
      // nonlinear outer loop had stopped before this solve (the state still
      // holds the previous inner solve, and every launch returned at once)
      collect_timing(pl, pl->ev_pending, k_base, st.outer_done ? 0 : st.done ? st.iters : k);
      pl->timing_bytes = pass_bytes(pl, pl->timing_kind, sizeof(T));
    }
    if (st.done || k > pl->opt.maxit + 1) break;
    if (m > 0 && k == next_ref) {         // every iteration so far did work
      refine_step<T>(pl, track_rho, false);
      next_ref += m;
    }
    // predicted iterations left: log-linear extrapolation of ||r||^2 between
    // two polls.  With a prior (first_n > 0: the solve restarts from a nearby
    // iterate) the first poll already extrapolates, from ||r_0||^2 at
    // iteration 0, and a poll without a usable rate (the residual having
    // risen) is followed by half the iterations done; a solve from scratch
    // waits for a rate between two polls, two chunks apart.
    const bool prior = first_n > 0;
    n = prior ? std::max(1, std::min(2 * chunk, st.iters / 2)) : 2 * chunk;
    const bool from_start = prior && prev_rr < 0.0;
    if (from_start) {
      prev_rr = st.rr0;
      prev_it = 0;
    }
    if (prev_rr > 0.0 && st.rr > 0.0 && st.iters > prev_it && st.rr < prev_rr) {
      const double rate = std::log(st.rr / prev_rr) / double(st.iters - prev_it);
      const double left = std::log(st.thr2 / st.rr) / rate;
      n = (int)std::ceil(std::max(1.0, left));
      // PCG's residual falls faster after its first iterations, so a rate
      // measured from iteration 0 overstates what is left: at most half the
      // iterations done, then a poll with a rate from two polls
      if (from_start) n = std::min(n, std::max(1, st.iters / 2));
      n = std::max(1, std::min(n, 8 * chunk));
    }
    prev_rr = st.rr;
    prev_it = st.iters;
  }
  if (track) refine_step<T>(pl, track_rho, true);   // phi from the source s
  return st;
}

template <typename T>
void reset_state(gps_plan* pl, double abs_thr, double rel_thr, int rel_from_b = 0) {
  Res<T>& R = pl->res<T>();
  Batch b{};
  b.n = 1;
  launch_reset_state<T>(R.tab, b, abs_thr, rel_thr, rel_from_b, pl->stream());
}

template <typename T>
void finish_info(gps_plan* pl, const SolveState& st, const double* rho, double* phi_out,
                 int total_iters) {
  Res<T>& R = pl->res<T>();
  const long long n = pl->npts();
  ck(hipMemcpyAsync(phi_out, R.slot().phi, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice,
                    pl->stream()));
  Batch b{};
  b.n = 1;
  launch_energy<T>(R.tab, b, rho, n, pl->stream());
  ck(hipGetLastError());
  // energy partials and the iteration history come back in one host wait
  const int groups = vec_groups(n);
  ck(hipMemcpyAsync(R.h_parts, R.slot().part_aux, (size_t)groups * 2 * sizeof(double),
                    hipMemcpyDeviceToHost, pl->stream()));
  const int nh = std::min(st.iters, R.hist_cap);
  pl->hist.assign((size_t)4 * nh, 0.0);
  if (nh > 0)
    ck(hipMemcpyAsync(pl->hist.data(), R.slot().hist, (size_t)4 * nh * sizeof(double),
                      hipMemcpyDeviceToHost, pl->stream()));
  ck(hipStreamSynchronize(pl->stream()));
  double e = 0.0;
  for (int i = 0; i < groups; ++i) e += R.h_parts[(size_t)i * 2];
  pl->info.energy = 0.5 * pl->g.h * pl->g.h * pl->g.h * e;
  pl->info.iterations = total_iters;
  pl->info.rnorm0 = std::sqrt(st.rr0);
  pl->info.rel_residual = st.rr0 > 0 ? std::sqrt(st.rr / st.rr0) : 0.0;
  pl->info.history_len = nh;
}

struct Electrolyte {
  bool present = false;
  bool linear = false;
  IonParams ip{};
  double kappa_coef = 0.0;
  int outer_maxit = 0;
};

template <typename T>
gps_status solve_impl(gps_plan* pl, const double* rho, const double* eps, double* phi,
                      double tol, const Electrolyte& el, const double* q_user) {
  const bool nonlinear = el.present && !el.linear;
  // source tracking (refinement, warm start): single PCG solves on invertible
  // vacuum solvers
  const bool track = !nonlinear && pl->bc != GPS_BC_PERIODIC &&
                     (pl->opt.refine_every > 0 || pl->opt.warm_start);
  ensure_res<T>(pl, nonlinear, track);
  Res<T>& R = pl->res<T>();
  // warm start from the resident source of the previous tracked solve
  const bool warm = track && pl->opt.warm_start && R.have_src;
  R.have_src = false;
  hipStream_t s = pl->stream();
  const long long n = pl->npts();
  const int periodic = pl->bc == GPS_BC_PERIODIC;
  Slot<T>& sl = R.slot();
  Batch b{};
  b.n = 1;
  // Algorithm SCPBimproved's inner threshold for outer step 1 (see below)
  double rho_norm = 0.0;
  if (nonlinear) {
    // ||rho|| is needed before the first reset: one reduction on the host
    launch_init<T>(R.tab, b, rho, eps, n, 0, s);
    ck(hipGetLastError());
    rho_norm = std::sqrt(read_sum<T>(pl, sl.part_init, vec_groups(n), 4, 3));
    reset_state<T>(pl, kFourPi * tol * rho_norm, 1e-2);
  } else {
    reset_state<T>(pl, 0.0, tol, warm ? 1 : 0);
  }
  launch_init<T>(R.tab, b, rho, eps, n, warm ? 1 : 0, s);
  if (nonlinear) launch_zero_ion<T>(R.tab, b, n, s);
  const double kcoef = (el.present && el.linear) ? el.kappa_coef : 0.0;
  if (q_user) {
    launch_qcopy<T>(R.tab, b, n, q_user, s);
  } else {
    const double* lap = nullptr;
    if (periodic) {
      spectral_laplacian<T>(pl);
      lap = R.lap64;
    }
    launch_qfield<T>(R.tab, b, pl->g, pl->opt.fd_order / 2, lap, kcoef, eps, el.ip.gamma,
                     el.ip.eps_bulk, s);
  }
  if (periodic && kcoef != 0.0) {
    const Geom& g = pl->g;
    launch_set_g0<T>(R.tab, b, n, 1.0 / ((double)g.Lx * g.Ly * g.Lz), s);
  }
  ck(hipGetLastError());
  std::memset(&pl->info, 0, sizeof(pl->info));
  if (!nonlinear) {
    // warm start: phi_0 = S^-1 G s and r_0 = b - A phi_0 from the kept source
    if (warm) refine_step<T>(pl, rho, false);
    const SolveState st = run_pcg<T>(pl, periodic && !el.present, track ? rho : nullptr);
    R.have_src = track && (st.status == GPS_OK || st.status == GPS_E_NOT_CONVERGED);
    finish_info<T>(pl, st, rho, phi, st.iters);
    pl->info.status = st.status;
    return (gps_status)st.status;
  }
  // Algorithm SCPBimproved.  After each inner solve the ionic update and the
  // outer decision run on the device (k_outer_decide: outer residual, stop
  // test, and the reset of the inner state for the next step), and the next
  // inner solve's first iterations are queued behind them without a host
  // round trip; its first poll also returns the outer decision.  When the
  // outer loop has stopped, those queued iterations find the inner state
  // stopped and return at once.
  int total = 0;
  SolveState st{};
  gps_status result = GPS_E_NOT_CONVERGED;
  double outer_res = 0.0;
  int outer = 1;
  const double abs_thr = kFourPi * tol * rho_norm;
  st = run_pcg<T>(pl, 0);
  for (int k = 1;; ++k) {
    outer = k;
    total += st.iters;
    if (st.status != GPS_OK) {
      result = (gps_status)st.status;
      break;
    }
    IonParams ip = el.ip;
    ip.eps = eps;
    launch_ion_update<T>(R.tab, b, n, ip, k == 1, s);
    launch_outer_decide<T>(R.tab, b, vec_groups(n), rho_norm, tol, abs_thr,
                           k + 1 <= 2 ? 1e-2 : 0.0, k == el.outer_maxit, s);
    ck(hipGetLastError());
    // inner solves of consecutive outer steps need similar iteration counts
    const SolveState next = run_pcg<T>(pl, 0, nullptr, std::max(1, st.iters - 1));
    outer_res = next.outer_res;
    if (next.outer_done) {
      result = (gps_status)next.outer_status;
      break;
    }
    st = next;
  }
  finish_info<T>(pl, st, rho, phi, total);
  pl->info.outer_iterations = outer;
  pl->info.outer_residual = outer_res;
  pl->info.status = result;
  return result;
}

// Algorithm SC and the PSD minimization (Sec. II.A), on the device: per step
// one vacuum solve (the plan's passes, bulk precision) of f = r/eps, the
// operator A v = -4 pi r + eps grad ln eps . grad v with the two inner
// products of the step, then the update phi += alpha v, r -= alpha A v (FP64)
// with alpha taken on the device from the operator's partials, and a
// one-work-group stop decision.  PSD takes Algorithm PCG's step with beta =
// 0, (v, r)/(v, A v), and stops on ||r||_2; its weighted variant takes the
// step that minimizes ||r/eps||_2, (A v, r/eps^2)/(A v, A v/eps^2), and stops
// on ||r/eps||_2.  SC is the same recurrence with the fixed steps -1/(4 pi)
// (first) and -eta/(4 pi), and its residual ||rho_iter_{k+1} - rho_iter_k||
// equals (eta/4 pi) ||r/eps|| at the current iterate.  Steps are captured as
// graphs of 8, 4, 2 and 1 steps over plan-owned buffers (eps and phi are
// copied in and out), replayed for a predicted number of steps between polls
// of the device state; steps after the stop decision return at once.
template <typename T>
void ensure_sc(gps_plan* pl) {
  ensure_res<T>(pl, false);
  gps_plan::ScRes& S = pl->sc;
  if (S.st) return;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  const long long n = pl->npts();
  const size_t nd = (size_t)n * sizeof(double);
  const int gv = vec_groups(n), gp = polarization_groups(pl->g);
  dalloc(&S.r, nd, &S.bytes);
  dalloc(&S.v, nd, &S.bytes);
  dalloc(&S.av, nd, &S.bytes);
  dalloc(&S.f, nd, &S.bytes);
  dalloc(&S.lne, nd, &S.bytes);
  dalloc(&S.eps, nd, &S.bytes);
  dalloc(&S.phi, nd, &S.bytes);
  dalloc(&S.part_op, (size_t)2 * gp * sizeof(double), &S.bytes);
  dalloc(&S.part, (size_t)2 * gv * sizeof(double), &S.bytes);
  dalloc(&S.st, sizeof(ScState), &S.bytes);
  if (hipHostMalloc(reinterpret_cast<void**>(&S.h_st), sizeof(ScState)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&S.h_part), (size_t)2 * gv * sizeof(double)) !=
          hipSuccess)
    throw NoMem{};
}

// u = G f with the bulk-precision passes, enqueued on stream s (no wait).
template <typename T>
void enqueue_vacuum(gps_plan* pl, const double* f, double* u, hipStream_t s) {
  Res<T>& R = pl->res<T>();
  const Geom& g = pl->g;
  cplx<T>* work = R.slot().work;
  XParams<T> xp = xparams<T>(pl, g.ny * g.nz, g.ny, g.nx, g.nx, (long long)g.Ly * g.Kx, g.nx);
  xp.in_real = f;
  xp.out_real = u;
  xp.work = work;
  launch_xfwd<T>(XF_REAL, xp, s);
  SParams<T> yf = sparams<T>(pl, 1, g.Ly, g.ny, g.Ly, g.nz * g.Kx, g.Kx, (long long)g.Ly * g.Kx,
                             g.Kx);
  yf.work = work;
  launch_strided<T>(ST_FWD, yf, s);
  SParams<T> zc = sparams<T>(pl, 2, g.Lz, g.nz, g.nz, g.Ly * g.Kx, g.Ly * g.Kx, 0,
                             (long long)g.Ly * g.Kx);
  zc.work = work;
  zc.table = pl->green<T>();
  launch_strided<T>(ST_CONV, zc, s);
  SParams<T> yi = sparams<T>(pl, 1, g.Ly, g.Ly, g.ny, g.nz * g.Kx, g.Kx, (long long)g.Ly * g.Kx,
                             g.Kx);
  yi.work = work;
  launch_strided<T>(ST_INV, yi, s);
  launch_xinv<T>(XI_REAL, xp, s);
}

template <typename T>
void enqueue_sc_step(gps_plan* pl, int paper_step, hipStream_t s) {
  gps_plan::ScRes& S = pl->sc;
  const long long n = pl->npts();
  enqueue_vacuum<T>(pl, S.f, S.v, s);
  // the operator launch also takes the previous step's stop decision
  launch_sc_operator(pl->g, pl->opt.fd_order / 2, paper_step, S.r, S.eps, S.lne, S.v, S.av,
                     S.part_op, &S.st->done, ScDecide{S.part, vec_groups(n), S.st}, s);
  launch_sc_advance(n, S.eps, S.phi, S.r, S.v, S.av, S.f, S.part_op, polarization_groups(pl->g),
                    S.part, S.st, s);
}

template <typename T>
void build_sc_graphs(gps_plan* pl, int paper_step) {
  gps_plan::ScRes& S = pl->sc;
  const int key = paper_step + 2 * (pl->opt.fd_order / 2) + 64 * (sizeof(T) == sizeof(float));
  if (S.graphs[0] && S.graph_key == key) return;
  for (hipGraphExec_t& g : S.graphs) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  if (!pl->cap_stream) ck(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (int i = 0; i < 4; ++i) {
    ck(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < S.graph_iters[i]; ++j) enqueue_sc_step<T>(pl, paper_step, pl->cap_stream);
    // the last step's decision, so that the state read between replays is current
    launch_sc_decide(ScDecide{S.part, vec_groups(pl->npts()), S.st}, pl->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(pl->cap_stream, &graph);
    if (e != hipSuccess) throw DevError{e};
    const hipError_t e2 = hipGraphInstantiate(&S.graphs[i], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) throw DevError{e2};
  }
  S.graph_key = key;
}

ScState read_sc_state(gps_plan* pl) {
  gps_plan::ScRes& S = pl->sc;
  ck(hipMemcpyAsync(S.h_st, S.st, sizeof(ScState), hipMemcpyDeviceToHost, pl->stream()));
  ck(hipStreamSynchronize(pl->stream()));
  return *S.h_st;
}

template <typename T>
gps_status sc_impl(gps_plan* pl, const double* rho, const double* eps, double* phi, double tol,
                   int method, double eta) {
  ensure_sc<T>(pl);
  gps_plan::ScRes& S = pl->sc;
  const long long n = pl->npts();
  hipStream_t s = pl->stream();
  const int paper_step = method == GPS_METHOD_PSD;
  build_sc_graphs<T>(pl, paper_step);
  const int max_steps = method == GPS_METHOD_SC ? pl->opt.maxit + 1 : pl->opt.maxit;
  launch_sc_begin(n, rho, eps, S.r, S.f, S.phi, S.eps, S.lne, S.part, S.st, method, eta, tol,
                  max_steps, s);
  ck(hipGetLastError());
  std::memset(&pl->info, 0, sizeof(pl->info));
  pl->hist.clear();
  ScState st = read_sc_state(pl);
  // steps before the next poll: log-linear extrapolation of the stopping norm
  auto norm2 = [&](const ScState& z) {
    return method == GPS_METHOD_PSD ? z.rr : z.ff;
  };
  auto thr2 = [&](const ScState& z) {
    if (method == GPS_METHOD_PSD) return z.thr_r * z.thr_r;
    if (method == GPS_METHOD_PSD_WEIGHTED) return z.thr_w * z.thr_w;
    const double t = z.thr_sc * kFourPi / z.eta;     // SC: on ||r/eps||
    return t * t;
  };
  int n_next = 4;
  double prev = -1.0;
  int prev_step = 0;
  while (!st.done && st.step <= max_steps + 8) {
    int left = n_next;
    for (int i = 0; i < 4; ++i)
      for (; left >= S.graph_iters[i]; left -= S.graph_iters[i])
        ck(hipGraphLaunch(S.graphs[i], s));
    st = read_sc_state(pl);
    if (st.done) break;
    n_next = 4;
    const double cur = norm2(st);
    if (prev > 0.0 && cur > 0.0 && cur < prev && st.step > prev_step) {
      const double rate = std::log(cur / prev) / double(st.step - prev_step);
      const double need = std::log(thr2(st) / cur) / rate;
      n_next = (int)std::ceil(std::max(1.0, need));
    }
    n_next = std::max(1, std::min(n_next, 32));
    prev = cur;
    prev_step = st.step;
  }
  launch_sc_energy(n, rho, S.phi, S.part, s);
  ck(hipGetLastError());
  ck(hipMemcpyAsync(phi, S.phi, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  const int gv = vec_groups(n);
  ck(hipMemcpyAsync(S.h_part, S.part, (size_t)2 * gv * sizeof(double), hipMemcpyDeviceToHost, s));
  ck(hipStreamSynchronize(s));
  double e = 0.0;
  for (int i = 0; i < gv; ++i) e += S.h_part[(size_t)2 * i];
  const gps_status status = st.done ? (gps_status)st.status : GPS_E_NOT_CONVERGED;
  pl->info.status = status;
  pl->info.iterations = st.iters;
  pl->info.rnorm0 = std::sqrt(st.rr0);
  pl->info.rel_residual = st.rr0 > 0.0 ? std::sqrt(st.rr / st.rr0) : 0.0;
  pl->info.energy = 0.5 * pl->g.h * pl->g.h * pl->g.h * e;
  return status;
}

gps_status parse_electrolyte(const gps_plan* pl, const gps_ions* ions, Electrolyte* out) {
  if (ions->nspecies < 1 || ions->nspecies > 4 || !ions->Z || !ions->c_bulk) return GPS_E_INVALID;
  if (!(ions->kT > 0.0)) return GPS_E_INVALID;
  if (!ions->gamma && !(ions->eps_bulk > 1.0)) return GPS_E_INVALID;
  Electrolyte el;
  el.present = true;
  el.linear = ions->linear != 0;
  IonParams& ip = el.ip;
  ip.nspecies = ions->nspecies;
  ip.kT = ions->kT;
  ip.eta = ions->eta;
  ip.eps_bulk = ions->eps_bulk;
  ip.gamma = ions->gamma;
  ip.steric = ions->c_max != nullptr;
  double z2c = 0.0;
  for (int i = 0; i < ions->nspecies; ++i) {
    const double c = ions->c_bulk[i];
    if (!(c > 0.0) || !std::isfinite(ions->Z[i])) return GPS_E_INVALID;
    ip.Z[i] = ions->Z[i];
    ip.c[i] = c;
    ip.a[i] = 0.0;
    if (ip.steric) {
      const double cm = ions->c_max[i];
      if (!(cm > c)) return GPS_E_INVALID;
      ip.a[i] = c / cm;
    }
    z2c += ions->Z[i] * ions->Z[i] * c;
  }
  el.kappa_coef = kFourPi / ions->kT * z2c;
  if (!el.linear) {
    if (!(ions->eta > 0.0 && ions->eta <= 1.0) || ions->outer_maxit < 1) return GPS_E_INVALID;
    if (pl->bc == GPS_BC_PERIODIC) return GPS_E_UNSUPPORTED;
    el.outer_maxit = ions->outer_maxit;
  }
  *out = el;
  return GPS_OK;
}

// ---------------------------------------------------------------------------
// continuous batching (gps_batch.h)
// ---------------------------------------------------------------------------
template <typename T>
void ensure_batch(gps_plan* pl, int K) {
  ensure_res<T>(pl, false);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  Res<T>& R = pl->res<T>();
  if (R.nslots < K) {
    for (int i = R.nslots; i < K; ++i) {
      Slot<T>& sl = R.slot(i);
      sl = Slot<T>{};
      R.nslots = i + 1;            // free_res frees it even if an allocation below fails
      alloc_slot<T>(pl, sl, &R.bytes);
      dalloc(&sl.hist, (size_t)4 * R.hist_cap * sizeof(double), &R.bytes);
      sl.hist_cap = R.hist_cap;
      sl.maxit = pl->opt.maxit;
    }
    drop_graphs(R);                // the slot table changed
  }
  if (!R.h_states &&
      hipHostMalloc(reinterpret_cast<void**>(&R.h_states), kArgSlots * sizeof(SolveState)) !=
          hipSuccess) {
    R.h_states = nullptr;
    throw NoMem{};
  }
}

template <typename T>
void build_batch_graphs(gps_plan* pl, int K, int check_neutral, int chunk) {
  Res<T>& R = pl->res<T>();
  if (R.bgraphs[0] && R.bgraph_n == K && R.bgraph_neutral == check_neutral &&
      R.bgraph_chunk == chunk)
    return;
  for (hipGraphExec_t& g : R.bgraphs) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  if (!pl->cap_stream) ck(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
  Batch b{};
  b.n = K;
  for (int i = 0; i < K; ++i) b.slot[i] = i;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  const int sizes[Res<T>::kGraphs] = {4 * chunk, 2 * chunk, chunk, 4, 2, 1};
  for (int i = 0; i < Res<T>::kGraphs; ++i) {
    R.bgraph_iters[i] = sizes[i];
    ck(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < sizes[i]; ++j)
      enqueue_iteration<T>(pl, R.tab, b, check_neutral, pl->cap_stream, j, 0);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(pl->cap_stream, &graph);
    if (e != hipSuccess) throw DevError{e};
    const hipError_t e2 = hipGraphInstantiate(&R.bgraphs[i], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) throw DevError{e2};
  }
  R.bgraph_n = K;
  R.bgraph_neutral = check_neutral;
  R.bgraph_chunk = chunk;
}

template <typename T>
void batch_open_impl(gps_plan* pl, int K, int check_neutral) {
  ensure_batch<T>(pl, K);
  build_batch_graphs<T>(pl, K, check_neutral, pl->opt.check_every);
  Res<T>& R = pl->res<T>();
  Batch b{};
  b.n = K;
  for (int i = 0; i < K; ++i) b.slot[i] = i;
  launch_idle_state<T>(R.tab, b, pl->stream());
  ck(hipGetLastError());
  ck(hipStreamSynchronize(pl->stream()));
}

template <typename T>
void batch_join_impl(gps_plan* pl, int j, const BatchJoin& q, const Electrolyte& el) {
  Res<T>& R = pl->res<T>();
  hipStream_t s = pl->stream();
  const long long n = pl->npts();
  const int periodic = pl->bc == GPS_BC_PERIODIC;
  Batch b{};
  b.n = 1;
  b.slot[0] = j;
  launch_reset_state<T>(R.tab, b, 0.0, q.tol, 0, s);
  launch_init<T>(R.tab, b, q.rho, q.eps, n, 0, s);
  const double kcoef = el.present ? el.kappa_coef : 0.0;
  const double* lap = nullptr;
  if (periodic) {
    spectral_laplacian<T>(pl, j);
    lap = R.lap64;
  }
  launch_qfield<T>(R.tab, b, pl->g, pl->opt.fd_order / 2, lap, kcoef, q.eps, el.ip.gamma,
                   el.ip.eps_bulk, s);
  if (periodic && kcoef != 0.0) {
    const Geom& g = pl->g;
    launch_set_g0<T>(R.tab, b, n, 1.0 / ((double)g.Lx * g.Ly * g.Lz), s);
  }
  ck(hipGetLastError());
}

template <typename T>
void batch_advance_impl(gps_plan* pl, int iters, BatchSlot* out) {
  Res<T>& R = pl->res<T>();
  hipStream_t s = pl->stream();
  int left = iters;
  for (int i = 0; i < Res<T>::kGraphs; ++i)
    for (; left >= R.bgraph_iters[i]; left -= R.bgraph_iters[i])
      ck(hipGraphLaunch(R.bgraphs[i], s));
  const int K = R.bgraph_n;
  for (int i = 0; i < K; ++i)
    ck(hipMemcpyAsync(R.h_states + i, R.slot(i).st, sizeof(SolveState), hipMemcpyDeviceToHost,
                      s));
  ck(hipStreamSynchronize(s));
  for (int i = 0; i < K; ++i) {
    const SolveState& st = R.h_states[i];
    out[i] = BatchSlot{st.done, st.status, st.iters, st.rr, st.thr2, st.rr0};
  }
}

template <typename T>
double batch_finish_impl(gps_plan* pl, int j, const double* rho, double* phi) {
  Res<T>& R = pl->res<T>();
  hipStream_t s = pl->stream();
  const long long n = pl->npts();
  Batch b{};
  b.n = 1;
  b.slot[0] = j;
  ck(hipMemcpyAsync(phi, R.slot(j).phi, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_energy<T>(R.tab, b, rho, n, s);
  ck(hipGetLastError());
  const int groups = vec_groups(n);
  ck(hipMemcpyAsync(R.h_parts, R.slot(j).part_aux, (size_t)groups * 2 * sizeof(double),
                    hipMemcpyDeviceToHost, s));
  ck(hipStreamSynchronize(s));
  double e = 0.0;
  for (int i = 0; i < groups; ++i) e += R.h_parts[(size_t)i * 2];
  return 0.5 * pl->g.h * pl->g.h * pl->g.h * e;
}

}  // namespace


// ===========================================================================
// continuous batching entry points (internal API, gps_batch.h)
// ===========================================================================
namespace gps {

template <typename F>
static gps_status batch_guard(gps_plan* pl, F&& f) {
  pl->info.device_error = 0;
  try {
    f();
  } catch (const NoMem&) {
    return GPS_E_NOMEM;
  } catch (const DevError& d) {
    pl->info.device_error = (int)d.e;
    return GPS_E_DEVICE;
  }
  return GPS_OK;
}

static int batch_width(gps_plan* pl) {
  return pl->opt.precision == GPS_PREC_MIXED ? pl->res<float>().bgraph_n
                                             : pl->res<double>().bgraph_n;
}

gps_status batch_open(gps_plan* pl, int nslots, int check_neutral) {
  if (!pl || nslots < 1 || nslots > kArgSlots) return GPS_E_INVALID;
  if (pl->opt.refine_every > 0 || pl->opt.warm_start) return GPS_E_INVALID;
  if (pl->timing_kind != GPS_K_NONE) return GPS_E_INVALID;
  const bool mixed = pl->opt.precision == GPS_PREC_MIXED;
  return batch_guard(pl, [&] {
    if (mixed) batch_open_impl<float>(pl, nslots, check_neutral);
    else batch_open_impl<double>(pl, nslots, check_neutral);
  });
}

gps_status batch_join(gps_plan* pl, int slot, const BatchJoin& q) {
  if (!pl || slot < 0 || slot >= batch_width(pl) || !q.rho || !q.eps || !(q.tol > 0.0) ||
      !std::isfinite(q.tol))
    return GPS_E_INVALID;
  Electrolyte el;
  if (q.ions) {
    const gps_status st = parse_electrolyte(pl, q.ions, &el);
    if (st != GPS_OK) return st;
    if (!el.linear) return GPS_E_INVALID;
  }
  const bool mixed = pl->opt.precision == GPS_PREC_MIXED;
  return batch_guard(pl, [&] {
    if (mixed) batch_join_impl<float>(pl, slot, q, el);
    else batch_join_impl<double>(pl, slot, q, el);
  });
}

gps_status batch_advance(gps_plan* pl, int iters, BatchSlot* out) {
  if (!pl || iters < 1 || !out || batch_width(pl) < 1) return GPS_E_INVALID;
  const bool mixed = pl->opt.precision == GPS_PREC_MIXED;
  return batch_guard(pl, [&] {
    if (mixed) batch_advance_impl<float>(pl, iters, out);
    else batch_advance_impl<double>(pl, iters, out);
  });
}

gps_status batch_finish(gps_plan* pl, int slot, const double* rho, double* phi,
                        double* energy) {
  if (!pl || slot < 0 || slot >= batch_width(pl) || !rho || !phi || !energy)
    return GPS_E_INVALID;
  const bool mixed = pl->opt.precision == GPS_PREC_MIXED;
  return batch_guard(pl, [&] {
    *energy = mixed ? batch_finish_impl<float>(pl, slot, rho, phi)
                    : batch_finish_impl<double>(pl, slot, rho, phi);
  });
}

}  // namespace gps

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* gps_status_string(int st) {
  switch (st) {
    case GPS_OK: return "ok";
    case GPS_E_INVALID: return "invalid argument";
    case GPS_E_NOMEM: return "out of device memory";
    case GPS_E_NOT_CONVERGED: return "not converged";
    case GPS_E_BREAKDOWN: return "PCG breakdown";
    case GPS_E_NONFINITE: return "non-finite value";
    case GPS_E_DEVICE: return "HIP runtime error";
    case GPS_E_UNSUPPORTED: return "unsupported size";
    case GPS_PENDING: return "pending";
    default: return "unknown status";
  }
}

static void plan_release(gps_plan* pl) {
  if (!pl) return;
  for (hipEvent_t e : pl->ev_pool) (void)hipEventDestroy(e);
  pl->ev_pool.clear();
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  pl->cap_stream = nullptr;
  free_res<float>(pl);
  free_res<double>(pl);
  for (int a = 0; a < 3; ++a) {
    dfree(pl->tw64[a]);
    dfree(pl->tw32[a]);
  }
  dfree(pl->green64);
  dfree(pl->green32);
  dfree(pl->lap64t);
  dfree(pl->lap32t);
  dfree(pl->pol_lne);
  pl->pol_bytes = 0;
  free_sc(pl);
}

gps_status gps_plan_create(int nx, int ny, int nz, double h, int bc, gps_plan** out) {
  if (!out) return GPS_E_INVALID;
  *out = nullptr;
  if (nx < 2 || ny < 2 || nz < 2 || !(h > 0.0) || !std::isfinite(h)) return GPS_E_INVALID;
  if (bc != GPS_BC_FREE && bc != GPS_BC_SURFACE && bc != GPS_BC_PERIODIC && bc != GPS_BC_WIRE)
    return GPS_E_INVALID;
  gps_plan* pl = new (std::nothrow) gps_plan();
  if (!pl) return GPS_E_NOMEM;
  pl->bc = bc;
  pl->opt.precision = GPS_PREC_FP64;
  pl->opt.fd_order = 16;
  pl->opt.maxit = 1000;
  pl->opt.check_every = 4;
  pl->opt.stream = nullptr;
  pl->opt.refine_every = 0;
  pl->opt.warm_start = 0;
  Geom& g = pl->g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.h = h;
  g.periodic_x = bc == GPS_BC_SURFACE || bc == GPS_BC_PERIODIC;
  g.periodic_y = g.periodic_x;
  g.periodic_z = bc == GPS_BC_PERIODIC || bc == GPS_BC_WIRE;
  g.Lx = g.periodic_x ? nx : 2 * nx;
  g.Ly = g.periodic_y ? ny : 2 * ny;
  g.Lz = g.periodic_z ? nz : 2 * nz;
  g.Kx = g.Lx / 2 + 1;
  const int L[3] = {g.Lx, g.Ly, g.Lz};
  for (int a = 0; a < 3; ++a) {
    if (!factorize(L[a], &pl->rp[a])) {
      delete pl;
      return GPS_E_UNSUPPORTED;
    }
  }
  std::lock_guard<std::mutex> lk(g_plan_mu);
  try {
    if (hipGetDevice(&pl->device) != hipSuccess) throw DevError{hipErrorNoDevice};
    // plan-time work runs on the plan's own non-blocking stream, never on the
    // legacy null stream (which would synchronize with other threads' streams)
    ck(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
    std::vector<double> t64[3];
    std::vector<float> t32[3];
    for (int a = 0; a < 3; ++a) {
      t64[a].resize(2 * (size_t)L[a]);
      t32[a].resize(2 * (size_t)L[a]);
      for (int m = 0; m < L[a]; ++m) {
        const double ang = 2.0 * kPi * (double)m / (double)L[a];
        t64[a][2 * m] = std::cos(ang);
        t64[a][2 * m + 1] = -std::sin(ang);
        t32[a][2 * m] = (float)t64[a][2 * m];
        t32[a][2 * m + 1] = (float)t64[a][2 * m + 1];
      }
      dalloc(&pl->tw64[a], t64[a].size() * sizeof(double), &pl->bytes);
      dalloc(&pl->tw32[a], t32[a].size() * sizeof(float), &pl->bytes);
      ck(hipMemcpyAsync(pl->tw64[a], t64[a].data(), t64[a].size() * sizeof(double),
                        hipMemcpyHostToDevice, pl->cap_stream));
      ck(hipMemcpyAsync(pl->tw32[a], t32[a].data(), t32[a].size() * sizeof(float),
                        hipMemcpyHostToDevice, pl->cap_stream));
    }
    build_green(pl);   // synchronizes cap_stream (the host twiddles outlive the copies)
  } catch (const NoMem&) {
    plan_release(pl);
    delete pl;
    return GPS_E_NOMEM;
  } catch (const DevError&) {
    plan_release(pl);
    delete pl;
    return GPS_E_DEVICE;
  }
  *out = pl;
  return GPS_OK;
}

gps_status gps_plan_set_options(gps_plan* pl, const gps_options* o) {
  if (!pl || !o) return GPS_E_INVALID;
  if (o->precision != GPS_PREC_FP64 && o->precision != GPS_PREC_MIXED) return GPS_E_INVALID;
  if (o->fd_order < 2 || o->fd_order > 16 || (o->fd_order & 1)) return GPS_E_INVALID;
  if (o->maxit < 1 || o->check_every < 1) return GPS_E_INVALID;
  if (o->refine_every < 0 ||
      ((o->refine_every > 0 || o->warm_start) && pl->bc == GPS_BC_PERIODIC))
    return GPS_E_INVALID;
  pl->opt = *o;
  return GPS_OK;
}

gps_status gps_plan_get_options(const gps_plan* pl, gps_options* o) {
  if (!pl || !o) return GPS_E_INVALID;
  *o = pl->opt;
  return GPS_OK;
}

size_t gps_plan_device_bytes(const gps_plan* pl) {
  return pl ? pl->bytes + pl->r32.bytes + pl->r64.bytes + pl->pol_bytes + pl->sc.bytes : 0;
}

gps_status gps_plan_release_buffers(gps_plan* pl) {
  if (!pl) return GPS_E_INVALID;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  free_res<float>(pl);
  free_res<double>(pl);
  dfree(pl->pol_lne);
  pl->pol_bytes = 0;
  free_sc(pl);
  return GPS_OK;
}

gps_status gps_plan_footprint(int nx, int ny, int nz, int bc, int precision, int maxit,
                              int nonlinear_pb, int refine, size_t* tables, size_t* buffers,
                              size_t* transient) {
  if (nx < 2 || ny < 2 || nz < 2 || maxit < 1) return GPS_E_INVALID;
  if (bc != GPS_BC_FREE && bc != GPS_BC_SURFACE && bc != GPS_BC_PERIODIC && bc != GPS_BC_WIRE)
    return GPS_E_INVALID;
  if (precision != GPS_PREC_FP64 && precision != GPS_PREC_MIXED) return GPS_E_INVALID;
  // the same sizes as gps_plan_create, build_green and ensure_res
  const bool px = bc == GPS_BC_SURFACE || bc == GPS_BC_PERIODIC;   // x and y periodic
  const bool pz = bc == GPS_BC_PERIODIC;                           // fully periodic
  const bool zper = pz || bc == GPS_BC_WIRE;                      // z periodic
  const size_t Lx = px ? nx : 2 * (size_t)nx, Ly = px ? ny : 2 * (size_t)ny;
  const size_t Lz = zper ? nz : 2 * (size_t)nz, Kx = Lx / 2 + 1;
  const size_t n = (size_t)nx * ny * nz;
  const size_t s = precision == GPS_PREC_MIXED ? sizeof(float) : sizeof(double);
  const size_t ntab = (Lz / 2 + 1) * (Ly / 2 + 1) * Kx;
  const size_t nvg = (size_t)vec_groups((long long)n);
  const size_t nxg = ((size_t)ny * nz + 1) / 2 + 1;    // as part_caps
  const size_t wbox = (size_t)nz * Ly * Kx;
  size_t tb = 2 * (Lx + Ly + Lz) * (sizeof(double) + sizeof(float));         // twiddles
  tb += ntab * (sizeof(double) + sizeof(float));                              // Green table
  if (pz) tb += ntab * (sizeof(double) + sizeof(float));                      // Laplacian table
  size_t b = 5 * n * s + (pz ? n * s : 0) + n * sizeof(double);                     // vectors, sq64
  b += wbox * 2 * s;                                                          // work buffer
  const size_t nzg = Ly * Kx + 64;
  b += (4 * nvg + 3 * nxg + nzg + (size_t)kVec * nvg) * sizeof(double);         // partials
  b += sizeof(SolveState) + n * sizeof(double);                               // state, phi
  if (pz) b += n * sizeof(double) + (s != sizeof(double) ? wbox * 2 * sizeof(double) : 0);
  b += 4 * ((size_t)maxit + 1) * sizeof(double);                              // history
  if (nonlinear_pb) b += n * s;                                               // ionic charge
  if (refine && !pz) b += 4 * n * sizeof(double) + wbox * 2 * sizeof(double);    // sigma, s, q, Gs, work
  size_t t = 0;
  if (bc == GPS_BC_FREE) t = Lz * Ly * Kx * 2 * sizeof(double);
  else if (bc == GPS_BC_WIRE) t = Lz * Ly * (Kx * 2 + Lx) * sizeof(double);
  else if (bc == GPS_BC_SURFACE) t = Kx * (Ly / 2 + 1) * Lz * 2 * sizeof(double);
  if (tables) *tables = tb;
  if (buffers) *buffers = b;
  if (transient) *transient = t;
  return GPS_OK;
}

void gps_plan_destroy(gps_plan* pl) {
  if (!pl) return;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  plan_release(pl);
  delete pl;
}

static gps_status run_guarded(gps_plan* pl, bool mixed, const double* rho, const double* eps,
                              double* phi, double tol, const Electrolyte& el,
                              const double* q_user = nullptr) {
  pl->info.device_error = 0;
  try {
    if (mixed) return solve_impl<float>(pl, rho, eps, phi, tol, el, q_user);
    return solve_impl<double>(pl, rho, eps, phi, tol, el, q_user);
  } catch (const NoMem&) {
    return GPS_E_NOMEM;
  } catch (const DevError& d) {
    pl->info.device_error = (int)d.e;
    pl->info.status = GPS_E_DEVICE;
    return GPS_E_DEVICE;
  }
}

gps_status gps_solve_generalized(gps_plan* pl, const double* rho, const double* eps, double* phi,
                                 double tol) {
  if (!pl || !rho || !eps || !phi || !(tol > 0.0) || !std::isfinite(tol)) return GPS_E_INVALID;
  Electrolyte el;
  return run_guarded(pl, pl->opt.precision == GPS_PREC_MIXED, rho, eps, phi, tol, el);
}

gps_status gps_solve_generalized_q(gps_plan* pl, const double* rho, const double* eps,
                                   const double* q, double* phi, double tol) {
  if (!pl || !rho || !eps || !q || !phi || !(tol > 0.0) || !std::isfinite(tol))
    return GPS_E_INVALID;
  if (pl->bc == GPS_BC_PERIODIC) return GPS_E_INVALID;
  Electrolyte el;
  return run_guarded(pl, pl->opt.precision == GPS_PREC_MIXED, rho, eps, phi, tol, el, q);
}

gps_status gps_solve_sc(gps_plan* pl, const double* rho, const double* eps, double* phi,
                        double tol, int method, double eta) {
  if (!pl || !rho || !eps || !phi || !(tol > 0.0) || !std::isfinite(tol)) return GPS_E_INVALID;
  if (method != GPS_METHOD_SC && method != GPS_METHOD_PSD && method != GPS_METHOD_PSD_WEIGHTED)
    return GPS_E_INVALID;
  if (method == GPS_METHOD_SC && !(eta > 0.0 && eta <= 1.0)) return GPS_E_INVALID;
  if (pl->bc == GPS_BC_PERIODIC) return GPS_E_INVALID;
  pl->info.device_error = 0;
  try {
    if (pl->opt.precision == GPS_PREC_MIXED) return sc_impl<float>(pl, rho, eps, phi, tol, method, eta);
    return sc_impl<double>(pl, rho, eps, phi, tol, method, eta);
  } catch (const NoMem&) {
    return GPS_E_NOMEM;
  } catch (const DevError& d) {
    pl->info.device_error = (int)d.e;
    pl->info.status = GPS_E_DEVICE;
    return GPS_E_DEVICE;
  }
}

gps_status gps_rigid_cavity(gps_plan* pl, int natoms, const double* atoms, double delta,
                            double eps0, double* eps, double* q) {
  if (!pl || natoms < 1 || !atoms || !eps || !(delta > 0.0) || !std::isfinite(delta) ||
      !(eps0 >= 1.0) || !std::isfinite(eps0))
    return GPS_E_INVALID;
  try {
    // the atom table is checked on the host (finite centres, radii > 0)
    std::vector<double> h((size_t)natoms * 4);
    ck(hipMemcpyAsync(h.data(), atoms, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                      pl->stream()));
    ck(hipStreamSynchronize(pl->stream()));
    for (int a = 0; a < natoms; ++a) {
      const double* at = &h[(size_t)a * 4];
      if (!std::isfinite(at[0]) || !std::isfinite(at[1]) || !std::isfinite(at[2]) ||
          !(at[3] > 0.0) || !std::isfinite(at[3]))
        return GPS_E_INVALID;
    }
    launch_rigid_cavity(pl->g, atoms, natoms, delta, eps0, eps, q, pl->stream());
    ck(hipGetLastError());
    ck(hipStreamSynchronize(pl->stream()));
  } catch (const DevError& d) {
    pl->info.device_error = (int)d.e;
    return GPS_E_DEVICE;
  }
  return GPS_OK;
}

gps_status gps_polarization_charge(gps_plan* pl, const double* rho, const double* eps,
                                   const double* phi, double* rho_pol) {
  if (!pl || !rho || !eps || !phi || !rho_pol) return GPS_E_INVALID;
  try {
    if (!pl->pol_lne) {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      dalloc(&pl->pol_lne, (size_t)pl->npts() * sizeof(double), &pl->pol_bytes);
    }
    launch_log_field(pl->npts(), eps, pl->pol_lne, pl->stream());
    launch_polarization(pl->g, pl->opt.fd_order / 2, rho, eps, pl->pol_lne, phi, rho_pol,
                        pl->stream());
    ck(hipGetLastError());
    ck(hipStreamSynchronize(pl->stream()));
  } catch (const NoMem&) {
    return GPS_E_NOMEM;
  } catch (const DevError& d) {
    pl->info.device_error = (int)d.e;
    return GPS_E_DEVICE;
  }
  return GPS_OK;
}

gps_status gps_polarization_charge_noalloc(gps_plan* pl, const double* rho, const double* eps,
                                           const double* phi, double* rho_pol) {
  if (!pl || !rho || !eps || !phi || !rho_pol) return GPS_E_INVALID;
  if (pl->npts() > GPS_NOALLOC_MAX_POINTS) return GPS_E_INVALID;
  static_assert(GPS_NOALLOC_MAX_POINTS == kNoAllocMaxPoints, "scratch size");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return GPS_E_DEVICE;
  if (prev != pl->device && hipSetDevice(pl->device) != hipSuccess) return GPS_E_DEVICE;
  gps_status status = GPS_OK;
  try {
    double* lne = nullptr;
    ck(noalloc_scratch(pl->device, &lne));
    launch_log_field(pl->npts(), eps, lne, pl->stream());
    launch_polarization(pl->g, pl->opt.fd_order / 2, rho, eps, lne, phi, rho_pol,
                        pl->stream());
    ck(hipGetLastError());
    ck(hipStreamSynchronize(pl->stream()));
  } catch (const DevError& d) {
    pl->info.device_error = (int)d.e;
    status = GPS_E_DEVICE;
  }
  if (prev != pl->device) (void)hipSetDevice(prev);
  return status;
}

gps_status gps_solve_pb(gps_plan* pl, const double* rho, const double* eps, const gps_ions* ions,
                        double* phi, double tol) {
  if (!pl || !rho || !eps || !phi || !ions || !(tol > 0.0) || !std::isfinite(tol))
    return GPS_E_INVALID;
  Electrolyte el;
  const gps_status st = parse_electrolyte(pl, ions, &el);
  if (st != GPS_OK) return st;
  return run_guarded(pl, pl->opt.precision == GPS_PREC_MIXED, rho, eps, phi, tol, el);
}


gps_status gps_solve_vacuum(gps_plan* pl, const double* f, double* u) {
  if (!pl || !f || !u) return GPS_E_INVALID;
  try {
    if (pl->opt.precision == GPS_PREC_MIXED) vacuum_apply<float>(pl, f, u);
    else vacuum_apply<double>(pl, f, u);
  } catch (const NoMem&) {
    return GPS_E_NOMEM;
  } catch (const DevError&) {
    return GPS_E_DEVICE;
  }
  return GPS_OK;
}

gps_status gps_plan_set_timing(gps_plan* pl, int kind) {
  if (!pl || kind < GPS_K_NONE || kind > GPS_K_XINV) return GPS_E_INVALID;
  pl->timing_kind = kind;
  pl->timing_ms = 0.0;
  pl->timing_launches = 0;
  pl->timing_bytes = 0.0;
  pl->ev_pending.clear();
  // graphs record into pooled events: rebuild them with the new timing
  drop_graphs(pl->r32);
  drop_graphs(pl->r64);
  pl->ev_used = 0;
  return GPS_OK;
}

gps_status gps_plan_timing(const gps_plan* pl, double* total_ms, long long* launches,
                           double* bytes_per_launch) {
  if (!pl) return GPS_E_INVALID;
  if (total_ms) *total_ms = pl->timing_ms;
  if (launches) *launches = pl->timing_launches;
  if (bytes_per_launch) *bytes_per_launch = pl->timing_bytes;
  return GPS_OK;
}

gps_status gps_last_info(const gps_plan* pl, gps_info* out) {
  if (!pl || !out) return GPS_E_INVALID;
  *out = pl->info;
  return GPS_OK;
}

gps_status gps_last_history(const gps_plan* pl, double* out, int max_entries) {
  if (!pl || !out || max_entries < 0) return GPS_E_INVALID;
  const int n = std::min(max_entries, pl->info.history_len);
  std::memcpy(out, pl->hist.data(), (size_t)4 * n * sizeof(double));
  return GPS_OK;
}

}  // extern "C"
