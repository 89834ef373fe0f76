/*
 * gps.h -- generalized Poisson / Poisson-Boltzmann solver for AMD MI355X (gfx950).
 *
 * Method: Fisicaro, Genovese, Andreussi, Marzari, Goedecker, "A generalized
 * Poisson and Poisson-Boltzmann solver for electrostatic environments",
 * J. Chem. Phys. 144, 014103 (2016), arXiv:1509.00680.
 *
 *   gps_solve_generalized  Eq. GPe  div(eps grad phi) = -4 pi rho, solved by
 *                          Algorithm PCG (Sec. II.B) with the preconditioner
 *                          of Eq. PCGdef (the vacuum Poisson solver scaled by
 *                          sqrt(eps)) and the operator identity of Eq. corr.
 *   gps_solve_pb           Eq. PBe with the ionic charge of Eqs. rhoions,
 *                          ionsconcPB / ionsconcMPB / maxconc (Sec. III):
 *                          linear regime through Eq. corrPB inside PCG,
 *                          nonlinear regime through Algorithm SCPBimproved.
 *
 * Units: Hartree atomic units (bohr, Ha, e).  phi in Ha/e, rho in e/bohr^3.
 *
 * Grid and layout: every field is a C array double[nz][ny][nx] (x fastest)
 * on an orthorhombic cell-centred grid of spacing h; point (i, j, k) is at
 * ((i - (nx-1)/2) h, (j - (ny-1)/2) h, (k - (nz-1)/2) h).
 *
 * Memory: every field pointer passed to a solve is a DEVICE pointer (HIP
 * global memory of the device current at gps_plan_create) holding
 * nx*ny*nz doubles.  The caller owns rho, eps, gamma and phi; the plan owns
 * every internal buffer and frees it in gps_plan_destroy.  Solves are
 * enqueued on the plan's stream (gps_options.stream, default: the null
 * stream) and return after the stream has finished them.
 *
 * Threading: a plan is not thread-safe; distinct plans are independent.
 *
 * Errors: functions return a gps_status; nothing throws across this ABI.
 * On GPS_E_NOT_CONVERGED / GPS_E_BREAKDOWN phi holds the last iterate and
 * gps_last_info describes the solve.
 */
#ifndef GPS_H
#define GPS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary conditions of the vacuum Poisson solver (Sec. II.C):
 *   FREE      isolated system, zero-padded (Hockney) convolution with the
 *             cell-averaged 1/|r| kernel;
 *   SURFACE   periodic along x and y, isolated along z;
 *   PERIODIC  periodic along x, y and z (rho must be neutral for Poisson);
 *   WIRE      periodic along z, isolated along x and y: per z mode kz the
 *             cell-averaged in-plane kernel 2 K0(|kz| rho) (kz != 0) or
 *             -2 ln(rho / Rw) (kz = 0, Rw = 2 h sqrt(nx^2 + ny^2), a constant
 *             shift that keeps the operator positive definite; it adds a
 *             constant times the charge per unit length to phi), zero-padded
 *             in x and y. */
typedef enum { GPS_BC_FREE = 0, GPS_BC_SURFACE = 1, GPS_BC_PERIODIC = 2,
               GPS_BC_WIRE = 3 } gps_bc;

/* Arithmetic of the bulk work (FFT passes and PCG vectors).  Inner products,
 * the solution accumulator, the Green's-function tables and the stencil are
 * FP64 in both modes. */
typedef enum { GPS_PREC_FP64 = 0, GPS_PREC_MIXED = 1 } gps_precision;

typedef enum {
  GPS_OK = 0,
  GPS_E_INVALID = 1,        /* bad argument, eps <= 0, non-neutral periodic rho */
  GPS_E_NOMEM = 2,          /* device allocation failed */
  GPS_E_NOT_CONVERGED = 3,  /* maxit (or outer_maxit) reached */
  GPS_E_BREAKDOWN = 4,      /* (v, r) <= 0 or (p, Ap) >= 0 in PCG */
  GPS_E_NONFINITE = 5,      /* NaN/Inf in the inputs or during the iteration */
  GPS_E_DEVICE = 6,         /* HIP runtime error */
  GPS_E_UNSUPPORTED = 7,    /* FFT length with a prime factor other than 2,3,5,7 or > 1024 */
  GPS_PENDING = 8           /* serving: the request is still queued or running */
} gps_status;

typedef struct gps_plan gps_plan;

typedef struct {
  int precision;     /* gps_precision, default GPS_PREC_FP64 */
  int fd_order;      /* even order of the central differences of q (2..16), default 16 */
  int maxit;         /* PCG iteration cap, default 1000 */
  int check_every;   /* base length (PCG iterations) of the replayed graphs, default 4;
                        between polls of the device state the host replays graphs of
                        4, 2 and 1 times this length and of 4, 2 and 1 iterations to
                        cover the predicted iteration count */
  void *stream;      /* hipStream_t the solves run on; NULL = null stream */
  int refine_every;  /* true-residual refinement every m PCG iterations (0 = off, the
                        default).  The iterate is kept as sqrt(eps) phi = G s with the
                        source s in FP64; every m iterations phi and the residual
                        b - A phi are recomputed in FP64 (one FP64 vacuum solve) and PCG
                        restarts from them; on exit phi is recomputed from s.  Free and
                        surface boundaries; applies to gps_solve_generalized and linear
                        gps_solve_pb (the nonlinear outer loop ignores it).  Costs three
                        FP64 grid vectors and an FP64 FFT work buffer per plan. */
  int warm_start;    /* 1: start each solve from the previous solve's iterate on this plan
                        (kept as its FP64 source s, so the starting residual b - A phi is
                        exact in FP64) when that solve tracked it (any solve with
                        warm_start or refine_every set, that ended with GPS_OK or
                        GPS_E_NOT_CONVERGED); the caller guarantees that eps, fd_order and
                        the electrolyte are those of that solve.  The relative tolerance
                        stays relative to ||4 pi rho||.  Same scope and buffers as
                        refine_every.  Default 0. */
} gps_options;

/* Electrolyte of Sec. III (Eqs. rhoions, ionsconcPB, ionsconcMPB, maxconc).
 * Z, c_bulk (bohr^-3) and c_max (bohr^-3) are HOST arrays of nspecies
 * (1..4) entries; c_max NULL selects the Boltzmann law, otherwise the steric
 * law with the bracket read as (exp(-Z_j phi/kT) - 1).  gamma is a DEVICE
 * field in [0, 1] (ion accessibility); NULL selects (eps - 1)/(eps_bulk - 1).
 * linear != 0 solves the linear regime (Eq. corrPB: kappa2 =
 * (4 pi/kT) sum_i Z_i^2 c_i gamma inside PCG); otherwise Algorithm
 * SCPBimproved with mixing eta and at most outer_maxit outer steps. */
typedef struct {
  int nspecies;
  const double *Z;
  const double *c_bulk;
  const double *c_max;
  double kT;           /* Ha */
  const double *gamma;
  double eps_bulk;
  int linear;
  double eta;
  int outer_maxit;
} gps_ions;

typedef struct {
  int status;            /* gps_status of the last solve */
  int iterations;        /* PCG iterations (sum over outer steps for nonlinear PB) */
  int outer_iterations;  /* nonlinear PB outer steps, 0 otherwise */
  int history_len;       /* entries available through gps_last_history */
  double rnorm0;         /* ||r_0||_2 = ||4 pi rho||_2 */
  double rel_residual;   /* final ||r||_2 / ||r_0||_2 of the (last) PCG solve */
  double energy;         /* (1/2) h^3 sum rho phi */
  double outer_residual; /* ||rho^ions_k - rho^ions_{k-1}||_2 / ||rho||_2 (nonlinear PB) */
  int device_error;      /* hipError_t of the HIP call that failed (GPS_E_DEVICE), else 0 */
} gps_info;

/* Create a plan for an nx x ny x nz grid of spacing h (bohr) and boundary
 * condition bc.  Computes the Green's-function spectrum on the device (FP64)
 * and allocates the work buffers.  Errors: GPS_E_INVALID (n < 2, h <= 0 or
 * not finite, unknown bc, out == NULL), GPS_E_UNSUPPORTED (an FFT length
 * -- 2n on isolated axes, n on periodic axes -- with a prime factor > 7 or
 * longer than 1024), GPS_E_NOMEM, GPS_E_DEVICE.  *out is NULL on error. */
gps_status gps_plan_create(int nx, int ny, int nz, double h, int bc, gps_plan **out);

/* Replace the plan's options (NULL fields keep defaults: see gps_options).
 * Errors: GPS_E_INVALID for an odd or out-of-range fd_order, maxit < 1,
 * check_every < 1, unknown precision, refine_every < 0, or refine_every > 0 or
 * warm_start on a periodic plan. */
gps_status gps_plan_set_options(gps_plan *plan, const gps_options *opt);
gps_status gps_plan_get_options(const gps_plan *plan, gps_options *opt);

/* Device bytes held by the plan (tables + work buffers of both precisions
 * allocated so far). */
size_t gps_plan_device_bytes(const gps_plan *plan);

/* Device bytes of a plan for an nx x ny x nz grid with boundary condition bc:
 * *tables, held from gps_plan_create to gps_plan_destroy (twiddles, Green's
 * spectrum); *buffers, the per-solve buffers that one solve in `precision`
 * with iteration cap maxit allocates (nonlinear_pb != 0: a nonlinear
 * Poisson-Boltzmann solve, which adds the ionic-charge field; refine != 0:
 * true-residual refinement or warm start on, which adds their FP64 buffers) and
 * gps_plan_release_buffers frees; *transient, held only while gps_plan_create
 * builds the Green's spectrum (FP64 padded spectrum for free and surface BC).
 * After one solve gps_plan_device_bytes reports *tables + *buffers.  Any
 * output pointer may be NULL.  Errors: GPS_E_INVALID (n < 2, maxit < 1,
 * unknown bc or precision). */
gps_status gps_plan_footprint(int nx, int ny, int nz, int bc, int precision, int maxit,
                              int nonlinear_pb, int refine, size_t *tables, size_t *buffers,
                              size_t *transient);

/* Free the plan's per-solve buffers (both precisions) and its captured
 * iteration graphs, keeping the tables; the next solve allocates them again.
 * Errors: GPS_E_INVALID (null plan). */
gps_status gps_plan_release_buffers(gps_plan *plan);

void gps_plan_destroy(gps_plan *plan);

/* Solve div(eps grad phi) = -4 pi rho (Eq. GPe) to ||r||_2 <= tol ||4 pi rho||_2
 * (Algorithm PCG; r the PCG residual).  rho, eps: device, read only;
 * phi: device, written.  Errors: GPS_E_INVALID (null pointer, tol <= 0,
 * eps <= 0 anywhere, periodic rho with |sum rho| > 1e-10 sum |rho|),
 * GPS_E_NONFINITE, GPS_E_NOT_CONVERGED, GPS_E_BREAKDOWN, GPS_E_DEVICE. */
gps_status gps_solve_generalized(gps_plan *plan, const double *rho, const double *eps,
                                 double *phi, double tol);

/* Solve the Poisson-Boltzmann problem (Eq. PBe) for electrolyte ions.
 * linear: tol as in gps_solve_generalized.  Nonlinear: Algorithm
 * SCPBimproved, stopping when ||rho^ions_k - rho^ions_{k-1}||_2 <= tol ||rho||_2;
 * each inner PCG stops at ||r||_2 <= 4 pi tol ||rho||_2, except the first two
 * outer steps which stop at 1e-2 of their initial residual.  Errors: as
 * gps_solve_generalized, plus GPS_E_INVALID for a bad electrolyte
 * (nspecies outside 1..4, kT <= 0, c <= 0, c_max <= c, eta outside (0, 1],
 * eps_bulk <= 1 when gamma is NULL), GPS_E_NONFINITE when the ionic
 * charge overflows (Boltzmann law at large |phi|/kT), and GPS_E_UNSUPPORTED
 * for a nonlinear law on a periodic plan (there the potential's constant,
 * which sets the net ionic charge, is fixed by nothing in the algorithm: each
 * inner solve drops the zero mode of its source). */
gps_status gps_solve_pb(gps_plan *plan, const double *rho, const double *eps,
                        const gps_ions *ions, double *phi, double tol);

/* Vacuum Poisson solver of the plan (Eq. SPe, Sec. II.C): u = G_bc f, i.e.
 * lap u = -4 pi f under the plan's boundary condition, with the plan's
 * Green's function (the preconditioner of every PCG iteration without the
 * sqrt(eps) scaling).  Arithmetic in the plan's bulk precision.  f, u:
 * device double[nz][ny][nx]; f is read, u written (they may not alias).
 * Periodic: the k = 0 component of f is dropped (u has zero mean).
 * Errors: GPS_E_INVALID (null pointer), GPS_E_NOMEM, GPS_E_DEVICE. */
gps_status gps_solve_vacuum(gps_plan *plan, const double *f, double *u);

/* As gps_solve_generalized, with the correction vector q of Eq. corr
 * (q = sqrt(eps) lap sqrt(eps), in bohr^-2) given by the caller instead of the
 * plan's finite-difference one: for instance the analytic q of
 * gps_rigid_cavity (Sec. IV.A: every field that depends on eps follows
 * analytically from the cavity).  q: device double[nz][ny][nx], read only,
 * rounded to the bulk precision like the computed q.  Free, surface and wire
 * boundaries: with periodic boundaries the operator annihilates constants
 * only for the q of the plan's spectral Laplacian.  Errors: as
 * gps_solve_generalized, plus GPS_E_INVALID for a null q or a periodic plan. */
gps_status gps_solve_generalized_q(gps_plan *plan, const double *rho, const double *eps,
                                   const double *q, double *phi, double tol);

/* Algorithm SC and the PSD minimization of Sec. II.A (the paper's
 * self-consistent scheme and steepest descent, against which Algorithm PCG is
 * compared), on the same discrete operator
 *   A phi = eps L_G phi + eps (grad_h ln eps) . grad_h phi,  L_G = -4 pi G^-1,
 * with central differences of the plan's fd_order for the gradients (ghosts
 * as for q).  PSD is Algorithm PCG with beta = 0 and the preconditioner of
 * Eq. PrePSD (eps lap v = -4 pi r, v = G(r/eps)), with A v = -4 pi r +
 * eps grad ln eps . grad v.  Its step, per method:
 *   GPS_METHOD_PSD           Algorithm PCG's alpha = (v, r)/(v, A v); stops at
 *                            ||r||_2 <= tol ||4 pi rho||_2; GPS_E_BREAKDOWN if
 *                            (v, A v) = 0.  A and P are not symmetric in this
 *                            form and this step does not contract on the
 *                            paper's Gaussian test or on molecules (the
 *                            relative residual stays near 1): such solves end
 *                            with GPS_E_NOT_CONVERGED at maxit.
 *   GPS_METHOD_PSD_WEIGHTED  alpha = (A v, r/eps^2)/(A v, A v/eps^2), the step
 *                            that minimizes ||r/eps||_2 along A v; stops at
 *                            ||r/eps||_2 <= tol ||4 pi rho/eps||_2;
 *                            GPS_E_BREAKDOWN if A v = 0.
 * SC (Eqs. remap, rhoiter, linear mixing eta in (0, 1]): the same recurrence
 * with the fixed steps -1/(4 pi) (first, the unmixed phi_0 = G(rho/eps)) and
 * -eta/(4 pi), which reproduces Algorithm SC's iterates; stops when
 * ||rho_iter_{k+1} - rho_iter_k||_2 <= tol ||rho||_2 (gps_info.iterations counts
 * SC iterations after phi_0).  eta is ignored by the PSD methods.
 * At most maxit iterations.  The vacuum solves run in the plan's bulk
 * precision, everything else in FP64; the host takes alpha and the stop
 * decision after each step.  rho, eps: device, read; phi: device, written.
 * Free, surface and wire boundaries.  Errors: GPS_E_INVALID (null pointer,
 * tol <= 0, unknown method, eta outside (0, 1] for SC, a periodic plan),
 * GPS_E_NOT_CONVERGED, GPS_E_BREAKDOWN, GPS_E_NONFINITE, GPS_E_NOMEM,
 * GPS_E_DEVICE. */
typedef enum { GPS_METHOD_SC = 0, GPS_METHOD_PSD = 1,
               GPS_METHOD_PSD_WEIGHTED = 2 } gps_sc_method;
gps_status gps_solve_sc(gps_plan *plan, const double *rho, const double *eps, double *phi,
                        double tol, int method, double eta);

/* Rigid cavity of Eq. RigCav (Sec. IV.A) on the plan's grid:
 *   eps(r) = (eps0 - 1) prod_i h(d_i, Delta; |r - R_i|) + 1,
 * h the erf switch of Eq. hfunc, and, when q is not NULL, its correction
 * vector q = sqrt(eps) lap sqrt(eps) evaluated analytically (product rule over
 * the atoms; at a grid point on an atom centre that atom's cusp contributes
 * h''(0) to the Laplacian and nothing to the gradient).  Separations along
 * periodic axes of the plan are minimum-image ones in the cell of n h.
 * atoms: DEVICE array of natoms x 4 doubles (X, Y, Z, d_i) in bohr, in the
 * grid's coordinates (the grid is centred on the origin); eps and q: device
 * double[nz][ny][nx], written.  FP64.  Runs on the plan's stream and returns
 * when it has finished.  Errors: GPS_E_INVALID (null plan, atoms or eps,
 * natoms < 1, Delta <= 0, eps0 < 1, a non-finite value, a radius <= 0),
 * GPS_E_DEVICE. */
gps_status gps_rigid_cavity(gps_plan *plan, int natoms, const double *atoms, double delta,
                            double eps0, double *eps, double *q);

/* Polarization charge of the dielectric for a potential phi (Eqs. rhoiter,
 * remap; Eq. rhopol with the sign that Eq. remap implies):
 *   rho_pol = (1/4 pi) grad ln eps . grad phi - (1 - 1/eps) rho,
 * so that lap phi = -4 pi (rho + rho_pol).  Gradients are central
 * differences of the plan's fd_order, with edge-replicated ghosts on free axes
 * and wrapped ones on periodic axes.  rho, eps, phi: device, read; rho_pol:
 * device, written; all double[nz][ny][nx].  FP64.  The first call allocates
 * a scratch field (ln eps, nx*ny*nz doubles) that the plan keeps until
 * gps_plan_release_buffers or gps_plan_destroy (counted by
 * gps_plan_device_bytes).  Runs on the plan's stream and returns when it has
 * finished.  Errors: GPS_E_INVALID (null pointer), GPS_E_NOMEM, GPS_E_DEVICE. */
gps_status gps_polarization_charge(gps_plan *plan, const double *rho, const double *eps,
                                   const double *phi, double *rho_pol);

/* As gps_polarization_charge, but allocates nothing: for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The ln eps field it needs lives in a
 * static device array of GPS_NOALLOC_MAX_POINTS doubles (32 MiB) that the
 * library holds on each GPU it runs on until the process ends; its device
 * address is looked up on the first call on each device.  Every call on a GPU
 * shares that GPU's array, so calls that overlap on one GPU (several host
 * threads, or plans on different streams) race and must be serialized by the
 * caller.  The result is bit for bit that of gps_polarization_charge.
 * Runs on the plan's stream and returns when it has finished.  Errors:
 * GPS_E_INVALID (null pointer, or a plan of more than GPS_NOALLOC_MAX_POINTS
 * grid points), GPS_E_DEVICE. */
#define GPS_NOALLOC_MAX_POINTS 4194304
gps_status gps_polarization_charge_noalloc(gps_plan *plan, const double *rho,
                                           const double *eps, const double *phi,
                                           double *rho_pol);

/* Information about the last solve of this plan. */
gps_status gps_last_info(const gps_plan *plan, gps_info *out);

/* Per-iteration history of the last PCG solve: for iteration k, out[4k+0] =
 * (v_k, r_k), out[4k+1] = beta_k, out[4k+2] = alpha_k, out[4k+3] = ||r_{k+1}||^2.
 * Copies min(max_entries, history_len) entries to the HOST array out;
 * returns GPS_E_INVALID for a null plan/out. */
gps_status gps_last_history(const gps_plan *plan, double *out, int max_entries);

/* Kernel timing (instrumentation for measurement).  kind selects one pass of
 * the PCG iteration; while it is set, every solve times each launch of
 * that pass: two HIP events bound to the launch on the plan's stream
 * (hipExtLaunchKernel) take the kernel's start and end timestamps, and the
 * elapsed times of the launches that did work (iterations before the stop
 * decision) are accumulated.
 * Untimed solves replay the iterations as captured HIP graphs; timed solves
 * launch the same kernels one by one (events inside a graph are not
 * readable), so a timed solve is slower end to end than an untimed one.
 * GPS_K_NONE switches timing off.  Setting a kind clears the totals.
 * Errors: GPS_E_INVALID (null plan, unknown kind). */
typedef enum {
  GPS_K_NONE = 0,
  GPS_K_XFWD = 1,       /* x pass: alpha, phi and r update of the previous iteration,
                           ||r||^2, r/sqrt(eps), pairwise real-to-complex */
  GPS_K_YFWD = 2,       /* y pass, forward */
  GPS_K_ZCONV = 3,      /* z pass: forward, times the Green's spectrum (and (v, r) by
                           Parseval), inverse */
  GPS_K_YINV = 4,       /* y pass, inverse; its first work-group takes the stop decision
                           and beta */
  GPS_K_XINV = 5        /* x pass: complex-to-real, v = u/sqrt(eps), A v (Eq. corr),
                           p, Ap update and (p, Ap) */
} gps_kernel_kind;
gps_status gps_plan_set_timing(gps_plan *plan, int kind);

/* Totals of the timed pass since the last gps_plan_set_timing: *total_ms
 * (sum of launch durations), *launches, and *bytes_per_launch, the pass's
 * algorithmic HBM bytes per launch (every input read once, every output
 * written once) for the precision of the last solve.  Any output pointer may
 * be NULL.  Errors: GPS_E_INVALID (null plan). */
gps_status gps_plan_timing(const gps_plan *plan, double *total_ms, long long *launches,
                           double *bytes_per_launch);

const char *gps_status_string(int status);

/* ---- serving ---------------------------------------------------------------
 * A server runs independent solves that arrive over time (continuous
 * batching).  Each request is a full problem of its own: grid, spacing,
 * boundary condition, fields and, optionally, an electrolyte.  max_active
 * worker threads each own a HIP stream (non-blocking, default priority) and
 * take the oldest waiting request as soon as they are free and it is
 * admitted.  The solves of different workers then run on the device at the
 * same time.  Plans (Green's spectrum, work buffers, captured iteration
 * graphs) stay resident between requests and are reused by any request of
 * the same nx, ny, nz, h and bc.
 *
 * Batched launches: generalized Poisson and linear Poisson-Boltzmann requests
 * on grids of at most 64^3 points (whose solves are bound by launch latency)
 * run in continuous batches.  Their plan holds batch_slots problems, and every
 * kernel of an iteration is one launch over all of them, each with its own
 * buffers, coefficients and device-side stop decision.  A waiting request of
 * the same plan (and, for periodic boundaries, the same kind) joins a free
 * slot between two replays of the captured iteration graphs, and a request
 * leaves as soon as the host reads its state as done; other workers leave such
 * requests to the running batch.  Larger grids and nonlinear Poisson-Boltzmann
 * requests get one solve per plan.
 *
 * Admission is by device footprint (gps_plan_footprint; a batched plan counts
 * batch_slots times the buffers of one solve).  A request is
 * admitted when the bytes that the server's plans hold, plus what its own solve
 * adds (new tables, buffers and the transient of a new plan; only the
 * buffers if a resident plan has released them), fit in budget_bytes.  To make
 * room, idle plans release their buffers (gps_plan_release_buffers) and then
 * are destroyed, least recently used first in both steps.  Otherwise the request waits until
 * a running solve finishes.  Requests are taken in arrival order, except that
 * a waiting request among the next 16 whose plan is resident and idle may go
 * ahead of older ones that need a new plan.  No request is passed over more
 * than 8 times.
 *
 * A result is the same whether its request runs alone or among others: each
 * problem has its own buffers and state, and the kernels reduce in a fixed
 * order that does not depend on the other problems of a launch.
 *
 * Fields are device pointers, as for the plan calls.  They must hold their
 * final values when gps_server_submit is called (the workers' streams do not
 * wait for work on the caller's streams).  The caller keeps rho, eps, phi (and
 * gamma) valid and unmodified until the request's result has been returned
 * by gps_server_poll or gps_server_wait; phi is complete by then. */
typedef struct gps_server gps_server;

typedef struct {
  size_t budget_bytes;  /* device bytes the server's plans may hold, transients
                           included; 0 = no limit */
  int max_active;       /* worker streams, 1..16 (default 4) */
  int precision;        /* gps_precision of every solve (default GPS_PREC_MIXED) */
  int fd_order;         /* as gps_options (default 16) */
  int maxit;            /* as gps_options (default 1000) */
  int batch_slots;      /* problems per batched launch on grids of at most 64^3
                           points, 1..8 (0 = default 4; 1 = no batching) */
} gps_server_options;

typedef struct {
  int nx, ny, nz;
  double h;
  int bc;
  const double *rho;    /* device, read */
  const double *eps;    /* device, read */
  double *phi;          /* device, written */
  const gps_ions *ions; /* NULL: generalized Poisson (gps_solve_generalized);
                           else Poisson-Boltzmann (gps_solve_pb).  The struct
                           and its host arrays are copied at submission. */
  double tol;
  unsigned long long eps_key;  /* 0, or the caller's identity of this request's
                           dielectric: requests with the same nonzero key
                           promise the same eps (bit for bit).  Warm-start cache:
                           such a request (free, surface or wire boundaries,
                           generalized Poisson or linear PB) runs on a plan that
                           keeps the FP64 source of its final iterate, and when
                           the last solve on that plan had the same key (and the
                           same electrolyte) it starts from that iterate
                           (gps_options.warm_start) instead of from phi = 0. */
} gps_request;

typedef struct {
  int status;            /* gps_status of the solve */
  int iterations;
  int outer_iterations;
  double rel_residual;
  double energy;
  double submit_ms;      /* server clock: ms since gps_server_create */
  double start_ms;       /* admitted and taken by a worker */
  double done_ms;        /* phi written and the worker's stream idle */
  int worker;            /* index of the worker that ran it */
  int plan_reused;       /* 1 if an existing resident plan served it */
  int device_error;      /* as gps_info.device_error */
  int warm_started;      /* 1 if it started from a cached iterate (eps_key) */
} gps_result;

typedef struct {
  size_t bytes_in_use;   /* resident plans plus admitted transients */
  size_t bytes_peak;
  int plans_resident;
  int plans_created;
  int plans_evicted;     /* destroyed to make room */
  int buffers_released;  /* idle plans whose buffers were released to make room */
  int max_in_flight;     /* largest number of solves running at once */
  long long submitted;
  long long completed;
  long long batched;     /* requests solved in a slot of a batched plan */
  int max_batch;         /* most problems in flight in one batched launch */
} gps_server_stats;

/* Start a server on the current device.  opt may be NULL (defaults).
 * Errors: GPS_E_INVALID (out NULL, max_active outside 1..16, bad precision,
 * fd_order or maxit), GPS_E_DEVICE. */
gps_status gps_server_create(const gps_server_options *opt, gps_server **out);

/* Queue a request; *ticket identifies it.  Errors: GPS_E_INVALID (null
 * pointers, n < 2, h <= 0, unknown bc, tol <= 0, ions with nspecies outside
 * 1..4 or null arrays), GPS_E_NOMEM (the request alone exceeds the budget).
 * Problems found while solving (bad electrolyte, eps <= 0, ...) are reported
 * in the result's status. */
gps_status gps_server_submit(gps_server *srv, const gps_request *req, long long *ticket);

/* GPS_PENDING while the request is queued or running.  GPS_OK once it has
 * finished: *out is filled and the ticket is released.  GPS_E_INVALID for an
 * unknown or released ticket. */
gps_status gps_server_poll(gps_server *srv, long long ticket, gps_result *out);

/* As gps_server_poll, but blocks until the request has finished. */
gps_status gps_server_wait(gps_server *srv, long long ticket, gps_result *out);

gps_status gps_server_get_stats(gps_server *srv, gps_server_stats *out);

/* Finish every submitted request, then free the plans and the workers. */
void gps_server_destroy(gps_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* GPS_H */
