// Continuous batching of PCG solves on one plan (internal; used by the
// serving loop).  A plan opened for a batch holds `nslots` problems, each with
// its own buffers and device-side solve state.  The iteration is captured once
// as graphs whose launches cover every slot (blockIdx.y); a slot whose state
// says done returns at once from every kernel.  Problems join a free slot
// between graph replays (their initialisation kernels are enqueued on the
// plan's stream) and leave when the host reads their state as done, so the
// set of problems in flight changes at graph boundaries only.  All calls run
// on the plan's stream; the plan must not be used by another thread meanwhile.
#pragma once

#include "gps.h"
#include "gps_internal.h"

namespace gps {

// Request of one slot: generalized Poisson (ions null) or linear
// Poisson-Boltzmann (ions->linear != 0); relative tolerance tol.
struct BatchJoin {
  const double* rho;
  const double* eps;
  const gps_ions* ions;
  double tol;
};

// Host copy of a slot's state after batch_advance.
struct BatchSlot {
  int done;           // the slot's solve has stopped (or the slot is free)
  int status;         // gps_status once done
  int iterations;     // iterations completed
  double rr;          // last ||r||^2
  double thr2;        // stop threshold on ||r||^2
  double rr0;         // ||r_0||^2
};

// Allocates nslots (1..kArgSlots) slots on the plan (bulk precision of its
// options) and captures the batch graphs; check_neutral: periodic generalized
// Poisson (input neutrality checked at the first decision).  Every slot
// starts free.  GPS_E_INVALID for a bad nslots or a plan with refinement or
// warm start on.
gps_status batch_open(gps_plan* pl, int nslots, int check_neutral);
// Starts a request in free slot `slot`.  GPS_E_INVALID for a bad slot or
// electrolyte (the checks of gps_solve_pb; nonlinear ions are rejected).
gps_status batch_join(gps_plan* pl, int slot, const BatchJoin& req);
// Replays `iters` iterations over all slots, then waits for the stream and
// copies every slot's state into out[0..nslots).
gps_status batch_advance(gps_plan* pl, int iters, BatchSlot* out);
// After a slot is done: phi (device, written) and the energy (1/2) h^3 sum rho
// phi; the slot becomes free.  rho is the request's charge density.
gps_status batch_finish(gps_plan* pl, int slot, const double* rho, double* phi,
                        double* energy);

}  // namespace gps
