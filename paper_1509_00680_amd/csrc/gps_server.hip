// Serving loop of libgps (include/gps.h, gps_server_*): independent solves
// that arrive over time run on a pool of worker threads, one HIP stream each,
// with plans kept resident between requests and admission by device
// footprint.  Host code only; every solve goes through the plan ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gps.h"
#include "gps_batch.h"

namespace {

using Clock = std::chrono::steady_clock;

// Admission: waiting requests examined for a resident idle plan, and how
// often the oldest request may be passed over for one of them.
constexpr int kLookahead = 16;
constexpr int kMaxBypass = 8;
// Grids of at most this many points are served in continuous batches (their
// solves are bound by launch latency, so one launch covering several of them
// costs about as much as one alone); larger grids get one solve per plan.
constexpr long long kBatchMaxPoints = 64LL * 64 * 64;
// PCG iterations per replayed graph in the serving plans.
constexpr int kServeChunk = 8;

struct PlanKey {
  int nx, ny, nz, bc;
  double h;
  bool operator==(const PlanKey& o) const {
    return nx == o.nx && ny == o.ny && nz == o.nz && bc == o.bc && h == o.h;
  }
};

// The electrolyte a cached iterate was computed with (none for Poisson).
struct IonSig {
  bool present = false;
  gps_ions ions{};
  double Z[4]{}, c[4]{}, cmax[4]{};
  bool operator==(const IonSig& o) const {
    if (present != o.present) return false;
    if (!present) return true;
    const gps_ions& a = ions;
    const gps_ions& b = o.ions;
    if (a.nspecies != b.nspecies || a.kT != b.kT || a.gamma != b.gamma ||
        a.eps_bulk != b.eps_bulk || a.linear != b.linear || (a.c_max == nullptr) != (b.c_max == nullptr))
      return false;
    for (int i = 0; i < a.nspecies; ++i)
      if (Z[i] != o.Z[i] || c[i] != o.c[i] || cmax[i] != o.cmax[i]) return false;
    return true;
  }
};

struct Request {
  long long ticket = 0;
  gps_request req{};
  PlanKey key{};
  bool tracked = false;    // eps_key given: warm-start cache
  IonSig sig{};
  bool batchable = false;  // small grid, generalized Poisson or linear PB
  int neutral = 0;         // periodic generalized Poisson (input neutrality checked)
  bool has_ions = false;
  gps_ions ions{};
  double Z[4]{}, c[4]{}, cmax[4]{};
  size_t tables = 0, buffers = 0, transient = 0;   // footprint (gps_plan_footprint)
  int bypassed = 0;                      // later requests admitted before it
  bool done = false;
  gps_result res{};
};

struct PlanEntry {
  gps_plan* plan = nullptr;
  PlanKey key{};
  size_t bytes = 0;
  bool busy = false;
  int batch_neutral = -1;  // while a batch runs on it: its neutrality class
  int free_slots = 0;      // while a batch runs on it: slots a request may join
  unsigned long long warm_key = 0;   // eps_key of the iterate the plan keeps (0: none)
  IonSig warm_sig{};
  bool released = false;   // buffers released (tables kept)
  unsigned long long last_use = 0;
};

}  // namespace

struct gps_server {
  gps_server_options opt{};
  int device = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work;   // a request arrived or memory / a plan was freed
  std::condition_variable cv_done;   // a request finished
  std::deque<Request*> queue;
  std::unordered_map<long long, Request*> reqs;
  std::vector<PlanEntry*> plans;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  long long next_ticket = 1;
  unsigned long long use_clock = 0;
  bool stopping = false;
  int in_flight = 0;
  gps_server_stats stats{};

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
  void charge(size_t b) {
    stats.bytes_in_use += b;
    stats.bytes_peak = std::max(stats.bytes_peak, stats.bytes_in_use);
  }
  void refund(size_t b) { stats.bytes_in_use -= std::min(b, stats.bytes_in_use); }

  // A running batch that request R can join at its next poll.
  bool joinable(const Request* R) const {
    if (!R->batchable) return false;
    for (const PlanEntry* e : plans)
      if (e->busy && e->key == R->key && e->batch_neutral == R->neutral && e->free_slots > 0)
        return true;
    return false;
  }
  // An idle resident plan for R: one that keeps R's cached iterate first,
  // else the most recently used.
  PlanEntry* idle_plan(const Request* R) {
    PlanEntry* best = nullptr;
    for (PlanEntry* e : plans) {
      if (e->busy || !(e->key == R->key)) continue;
      if (R->tracked && e->warm_key == R->req.eps_key && e->warm_sig == R->sig) return e;
      if (!best || e->last_use > best->last_use) best = e;
    }
    return best;
  }
  // Releases the buffers of the least recently used idle plan that holds
  // any (other than `keep`); false if there is none.
  bool release_one(const PlanEntry* keep) {
    PlanEntry* v = nullptr;
    for (PlanEntry* e : plans)
      if (!e->busy && e != keep && !e->released && (!v || e->last_use < v->last_use)) v = e;
    if (!v) return false;
    gps_plan_release_buffers(v->plan);
    v->warm_key = 0;                 // the cached iterate went with the buffers
    const size_t now = gps_plan_device_bytes(v->plan);
    refund(v->bytes - std::min(now, v->bytes));
    v->bytes = now;
    v->released = true;
    ++stats.buffers_released;
    return true;
  }
  // Destroys the least recently used idle plan (other than `keep`); false if
  // there is none.
  bool evict_one(const PlanEntry* keep) {
    auto it = plans.end();
    for (auto i = plans.begin(); i != plans.end(); ++i)
      if (!(*i)->busy && *i != keep && (it == plans.end() || (*i)->last_use < (*it)->last_use))
        it = i;
    if (it == plans.end()) return false;
    PlanEntry* e = *it;
    plans.erase(it);
    gps_plan_destroy(e->plan);
    refund(e->bytes);
    ++stats.plans_evicted;
    --stats.plans_resident;
    delete e;
    return true;
  }
  bool fits(size_t need) const {
    return opt.budget_bytes == 0 || stats.bytes_in_use + need <= opt.budget_bytes;
  }
  // Frees idle plans' memory until `need` more bytes fit: buffers first, then
  // whole plans, least recently used first.
  bool make_room(size_t need, const PlanEntry* keep) {
    while (!fits(need) && release_one(keep)) {
    }
    while (!fits(need) && evict_one(keep)) {
    }
    return fits(need);
  }
};

namespace {

// Creates plan e for `key` when e->plan is null and applies the server's
// options with stream st.  Called without the server lock.
gps_status prepare_plan(gps_server* S, PlanEntry* e, const PlanKey& key, hipStream_t st,
                        int warm_start = 0, int refine_every = 0) {
  gps_status status = GPS_OK;
  if (!e->plan) {
    status = gps_plan_create(key.nx, key.ny, key.nz, key.h, key.bc, &e->plan);
    if (status != GPS_OK) e->plan = nullptr;
  }
  if (status == GPS_OK) {
    gps_options o{};
    gps_plan_get_options(e->plan, &o);
    o.precision = S->opt.precision;
    o.fd_order = S->opt.fd_order;
    o.maxit = S->opt.maxit;
    o.check_every = kServeChunk;
    o.stream = st;
    o.warm_start = warm_start;
    o.refine_every = refine_every;
    status = gps_plan_set_options(e->plan, &o);
  }
  return status;
}

// Runs one admitted request on stream st with plan e (created here when
// e->plan is null).  Called without the server lock.
void run_request(gps_server* S, Request* R, PlanEntry* e, hipStream_t st) {
  // warm-start cache: a tracked request keeps the FP64 source of its iterate
  // (refine_every past maxit: tracked, never refined) and starts from the
  // plan's cached iterate when it was computed for the same eps and ions
  const bool warm = R->tracked && e->plan && e->warm_key == R->req.eps_key && e->warm_sig == R->sig;
  gps_status status = prepare_plan(S, e, R->key, st, warm ? 1 : 0,
                                   R->tracked && !warm ? S->opt.maxit + 1 : 0);
  R->res.warm_started = warm ? 1 : 0;
  e->warm_key = 0;
  if (status == GPS_OK) {
    const gps_request& q = R->req;
    status = R->has_ions ? gps_solve_pb(e->plan, q.rho, q.eps, &R->ions, q.phi, q.tol)
                         : gps_solve_generalized(e->plan, q.rho, q.eps, q.phi, q.tol);
    if (hipStreamSynchronize(st) != hipSuccess && status == GPS_OK) status = GPS_E_DEVICE;
    gps_info info{};
    gps_last_info(e->plan, &info);
    R->res.iterations = info.iterations;
    R->res.outer_iterations = info.outer_iterations;
    R->res.rel_residual = info.rel_residual;
    R->res.energy = info.energy;
    R->res.device_error = info.device_error;
    if (R->tracked && (status == GPS_OK || status == GPS_E_NOT_CONVERGED)) {
      e->warm_key = R->req.eps_key;
      e->warm_sig = R->sig;
    }
  }
  R->res.status = status;
}

// Marks request R finished (status and figures already in R->res).
void publish(gps_server* S, Request* R) {
  std::lock_guard<std::mutex> lk(S->mu);
  --S->in_flight;
  R->res.done_ms = S->now_ms();
  R->done = true;
  ++S->stats.completed;
  S->cv_done.notify_all();
}

// PCG iterations a slot is predicted to need before its stop decision:
// log-linear extrapolation of ||r||^2 from its last two polls.
int predict_iters(const gps::BatchSlot& b, double prev_rr, int prev_it) {
  int n = 2 * kServeChunk;
  if (prev_rr > 0.0 && b.rr > 0.0 && b.iterations > prev_it && b.rr < prev_rr) {
    const double rate = std::log(b.rr / prev_rr) / double(b.iterations - prev_it);
    const double left = std::log(b.thr2 / b.rr) / rate;
    n = (int)std::ceil(std::max(1.0, left));
  }
  return std::max(1, std::min(n, 8 * kServeChunk));
}

// Continuous batch on plan e, started with the admitted request `first`:
// requests of the same plan (and neutrality class) that wait in the queue
// join free slots between graph replays, and each request is published as
// soon as its slot's state says done.  Ends when no slot is busy and no such
// request waits.  Called without the server lock; publishes every request it
// took, `first` included.
void run_batch(gps_server* S, Request* first, PlanEntry* e, hipStream_t st, int w) {
  const int K = S->opt.batch_slots;
  e->warm_key = 0;                   // slot 0's initialisation clears a cached iterate
  gps_status status = prepare_plan(S, e, first->key, st);
  if (status == GPS_OK) status = gps::batch_open(e->plan, K, first->neutral);
  if (status != GPS_OK) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      e->free_slots = 0;
      e->batch_neutral = -1;
    }
    first->res.status = status;
    publish(S, first);
    return;
  }
  Request* slot[gps::kArgSlots] = {};
  double prev_rr[gps::kArgSlots] = {};
  int prev_it[gps::kArgSlots] = {};
  gps::BatchSlot info[gps::kArgSlots] = {};
  auto join = [&](int i, Request* R) {
    const gps::BatchJoin q{R->req.rho, R->req.eps, R->has_ions ? &R->ions : nullptr,
                           R->req.tol};
    const gps_status js = gps::batch_join(e->plan, i, q);
    if (js != GPS_OK) {
      R->res.status = js;
      publish(S, R);
      return;
    }
    slot[i] = R;
    prev_rr[i] = -1.0;
    prev_it[i] = 0;
    int busy = 0;
    for (int k = 0; k < K; ++k) busy += slot[k] != nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->stats.batched;
    S->stats.max_batch = std::max(S->stats.max_batch, busy);
    info[i] = gps::BatchSlot{0, 0, 0, -1.0, 0.0, 0.0};
  };
  Request* incoming[gps::kArgSlots] = {};
  incoming[0] = first;
  for (;;) {
    for (int i = 0; i < K; ++i)
      if (incoming[i]) {
        join(i, incoming[i]);
        incoming[i] = nullptr;
      }
    int active = 0;
    for (int i = 0; i < K; ++i) active += slot[i] != nullptr;
    if (active > 0) {
      int n = 8 * kServeChunk;
      for (int i = 0; i < K; ++i)
        if (slot[i]) n = std::min(n, predict_iters(info[i], prev_rr[i], prev_it[i]));
      for (int i = 0; i < K; ++i)
        if (slot[i]) {
          prev_rr[i] = info[i].rr;
          prev_it[i] = info[i].iterations;
        }
      status = gps::batch_advance(e->plan, n, info);
      for (int i = 0; i < K; ++i) {
        Request* R = slot[i];
        if (!R || (status == GPS_OK && !info[i].done)) continue;
        gps_status rs = status;
        if (rs == GPS_OK) {
          double energy = 0.0;
          rs = gps::batch_finish(e->plan, i, R->req.rho, R->req.phi, &energy);
          if (rs == GPS_OK) rs = (gps_status)info[i].status;
          R->res.iterations = info[i].iterations;
          R->res.energy = energy;
          R->res.rel_residual = info[i].rr0 > 0.0 ? std::sqrt(info[i].rr / info[i].rr0) : 0.0;
        }
        gps_info pi{};
        gps_last_info(e->plan, &pi);
        R->res.device_error = pi.device_error;
        R->res.status = rs;
        slot[i] = nullptr;
        publish(S, R);
      }
      if (status != GPS_OK) break;      // the plan's stream failed: end the batch
    }
    // waiting requests of this plan take the free slots
    std::lock_guard<std::mutex> lk(S->mu);
    int busy = 0;
    for (int i = 0; i < K; ++i) {
      if (slot[i]) {
        ++busy;
        continue;
      }
      auto it = std::find_if(S->queue.begin(), S->queue.end(), [&](const Request* q) {
        return q->batchable && q->key == e->key && q->neutral == first->neutral;
      });
      if (it == S->queue.end()) continue;
      Request* R = *it;
      S->queue.erase(it);
      R->res.start_ms = S->now_ms();
      R->res.worker = w;
      R->res.plan_reused = 1;
      ++S->in_flight;
      S->stats.max_in_flight = std::max(S->stats.max_in_flight, S->in_flight);
      incoming[i] = R;
      ++busy;
    }
    e->free_slots = K - busy;
    e->batch_neutral = busy ? first->neutral : -1;
    if (!busy) {
      e->free_slots = 0;
      break;
    }
  }
  // a failed batch leaves its waiting joiners (none taken after the failure)
  std::lock_guard<std::mutex> lk(S->mu);
  e->free_slots = 0;
  e->batch_neutral = -1;
}

void worker_main(gps_server* S, int w) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[w];
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    Request* R = nullptr;
    PlanEntry* e = nullptr;
    size_t reserved = 0;
    bool fresh = false;
    for (;;) {
      if (S->queue.empty()) {
        if (S->stopping) return;
        S->cv_work.wait(lk);
        continue;
      }
      // requests that a running batch of their plan takes at its next poll
      // are left to it
      size_t head = 0;
      while (head < S->queue.size() && S->joinable(S->queue[head])) ++head;
      if (head == S->queue.size()) {
        S->cv_work.wait(lk);
        continue;
      }
      // a waiting request whose plan is resident and idle goes first (no plan
      // build); the oldest request is passed over at most kMaxBypass times
      R = S->queue[head];
      e = S->idle_plan(R);
      if (!e && R->bypassed < kMaxBypass) {
        const size_t look = std::min(S->queue.size(), head + (size_t)kLookahead);
        size_t pick = head;
        for (size_t i = head + 1; i < look && !e; ++i) {
          if (S->joinable(S->queue[i])) continue;
          e = S->idle_plan(S->queue[i]);
          pick = i;
        }
        if (e) {
          for (size_t i = head; i < pick; ++i) ++S->queue[i]->bypassed;
          R = S->queue[pick];
        }
      }
      if (e) {
        const size_t full = R->tables + R->buffers;
        reserved = full > e->bytes ? full - e->bytes : 0;
        if (S->make_room(reserved, e) || !S->in_flight) break;
        e = nullptr;
      } else {
        reserved = R->tables + R->buffers + R->transient;
        if (S->make_room(reserved, nullptr)) {
          e = new (std::nothrow) PlanEntry();
          if (e) {
            e->key = R->key;
            fresh = true;
            S->plans.push_back(e);
            ++S->stats.plans_resident;
            break;
          }
        }
        if (!S->in_flight) {   // nothing will free memory: fail the request
          S->queue.erase(std::find(S->queue.begin(), S->queue.end(), R));
          R->res.status = GPS_E_NOMEM;
          R->res.start_ms = R->res.done_ms = S->now_ms();
          R->res.worker = w;
          R->done = true;
          ++S->stats.completed;
          S->cv_done.notify_all();
          continue;
        }
      }
      S->cv_work.wait(lk);
    }
    S->queue.erase(std::find(S->queue.begin(), S->queue.end(), R));
    e->busy = true;
    S->charge(reserved);
    ++S->in_flight;
    S->stats.max_in_flight = std::max(S->stats.max_in_flight, S->in_flight);
    R->res.start_ms = S->now_ms();
    R->res.worker = w;
    R->res.plan_reused = fresh ? 0 : 1;
    const bool batch = R->batchable;
    if (batch) {
      e->batch_neutral = R->neutral;
      e->free_slots = S->opt.batch_slots - 1;
    }
    lk.unlock();

    if (batch) {
      run_batch(S, R, e, st, w);       // publishes R and every request that joined
      R = nullptr;
    } else {
      run_request(S, R, e, st);
    }

    lk.lock();
    if (R) --S->in_flight;
    S->refund(reserved);
    if (e->plan) {
      if (fresh) ++S->stats.plans_created;
      const size_t now = gps_plan_device_bytes(e->plan);
      S->refund(e->bytes);
      e->bytes = now;
      S->charge(now);
      e->released = false;
      e->busy = false;
      e->last_use = ++S->use_clock;
    } else {                       // plan creation failed
      S->plans.erase(std::find(S->plans.begin(), S->plans.end(), e));
      --S->stats.plans_resident;
      delete e;
    }
    if (R) {
      R->res.done_ms = S->now_ms();
      R->done = true;
      ++S->stats.completed;
      S->cv_done.notify_all();
    }
    S->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

gps_status gps_server_create(const gps_server_options* opt, gps_server** out) {
  if (!out) return GPS_E_INVALID;
  *out = nullptr;
  gps_server_options o{};
  o.budget_bytes = 0;
  o.max_active = 4;
  o.precision = GPS_PREC_MIXED;
  o.fd_order = 16;
  o.maxit = 1000;
  o.batch_slots = 4;
  if (opt) o = *opt;
  if (o.batch_slots == 0) o.batch_slots = 4;
  if (o.max_active < 1 || o.max_active > 16) return GPS_E_INVALID;
  if (o.batch_slots < 1 || o.batch_slots > gps::kArgSlots) return GPS_E_INVALID;
  if (o.precision != GPS_PREC_FP64 && o.precision != GPS_PREC_MIXED) return GPS_E_INVALID;
  if (o.fd_order < 2 || o.fd_order > 16 || (o.fd_order & 1) || o.maxit < 1) return GPS_E_INVALID;
  gps_server* S = new (std::nothrow) gps_server();
  if (!S) return GPS_E_NOMEM;
  S->opt = o;
  S->t0 = Clock::now();
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return GPS_E_DEVICE;
  }
  for (int w = 0; w < o.max_active; ++w) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
      delete S;
      return GPS_E_DEVICE;
    }
    S->streams.push_back(st);
  }
  for (int w = 0; w < o.max_active; ++w) S->workers.emplace_back(worker_main, S, w);
  *out = S;
  return GPS_OK;
}

gps_status gps_server_submit(gps_server* S, const gps_request* q, long long* ticket) {
  if (!S || !q || !ticket) return GPS_E_INVALID;
  if (q->nx < 2 || q->ny < 2 || q->nz < 2 || !(q->h > 0.0) || !(q->tol > 0.0)) return GPS_E_INVALID;
  if (q->bc != GPS_BC_FREE && q->bc != GPS_BC_SURFACE && q->bc != GPS_BC_PERIODIC &&
      q->bc != GPS_BC_WIRE)
    return GPS_E_INVALID;
  if (!q->rho || !q->eps || !q->phi) return GPS_E_INVALID;
  Request* R = new (std::nothrow) Request();
  if (!R) return GPS_E_NOMEM;
  R->req = *q;
  R->key = PlanKey{q->nx, q->ny, q->nz, q->bc, q->h};
  if (q->ions) {
    const gps_ions& in = *q->ions;
    if (in.nspecies < 1 || in.nspecies > 4 || !in.Z || !in.c_bulk) {
      delete R;
      return GPS_E_INVALID;
    }
    R->has_ions = true;
    R->ions = in;
    for (int i = 0; i < in.nspecies; ++i) {
      R->Z[i] = in.Z[i];
      R->c[i] = in.c_bulk[i];
      if (in.c_max) R->cmax[i] = in.c_max[i];
    }
    R->ions.Z = R->Z;
    R->ions.c_bulk = R->c;
    R->ions.c_max = in.c_max ? R->cmax : nullptr;
    R->req.ions = &R->ions;
    R->sig.present = true;
    R->sig.ions = in;
    for (int i = 0; i < in.nspecies; ++i) {
      R->sig.Z[i] = R->Z[i];
      R->sig.c[i] = R->c[i];
      R->sig.cmax[i] = R->cmax[i];
    }
  }
  const int nonlinear = R->has_ions && !R->ions.linear;
  R->tracked = q->eps_key != 0 && q->bc != GPS_BC_PERIODIC && !nonlinear;
  if (gps_plan_footprint(q->nx, q->ny, q->nz, q->bc, S->opt.precision, S->opt.maxit, nonlinear,
                         R->tracked ? 1 : 0, &R->tables, &R->buffers, &R->transient) != GPS_OK) {
    delete R;
    return GPS_E_INVALID;
  }
  R->neutral = q->bc == GPS_BC_PERIODIC && !R->has_ions;
  R->batchable = S->opt.batch_slots > 1 && !nonlinear && !R->tracked &&
                 (long long)q->nx * q->ny * q->nz <= kBatchMaxPoints;
  if (R->batchable) R->buffers *= (size_t)S->opt.batch_slots;   // a plan of batch_slots slots
  if (S->opt.budget_bytes && R->tables + R->buffers + R->transient > S->opt.budget_bytes) {
    delete R;
    return GPS_E_NOMEM;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  R->ticket = S->next_ticket++;
  R->res.submit_ms = S->now_ms();
  S->reqs[R->ticket] = R;
  S->queue.push_back(R);
  ++S->stats.submitted;
  *ticket = R->ticket;
  S->cv_work.notify_all();
  return GPS_OK;
}

static gps_status take_result(gps_server* S, long long ticket, gps_result* out, bool block) {
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return GPS_E_INVALID;
  Request* R = it->second;
  if (block)
    while (!R->done) S->cv_done.wait(lk);
  if (!R->done) return GPS_PENDING;
  if (out) *out = R->res;
  S->reqs.erase(it);
  delete R;
  return GPS_OK;
}

gps_status gps_server_poll(gps_server* S, long long ticket, gps_result* out) {
  if (!S) return GPS_E_INVALID;
  return take_result(S, ticket, out, false);
}

gps_status gps_server_wait(gps_server* S, long long ticket, gps_result* out) {
  if (!S) return GPS_E_INVALID;
  return take_result(S, ticket, out, true);
}

gps_status gps_server_get_stats(gps_server* S, gps_server_stats* out) {
  if (!S || !out) return GPS_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  return GPS_OK;
}

void gps_server_destroy(gps_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
    S->cv_work.notify_all();
  }
  for (std::thread& t : S->workers) t.join();
  for (PlanEntry* e : S->plans) {
    gps_plan_destroy(e->plan);
    delete e;
  }
  for (auto& kv : S->reqs) delete kv.second;
  for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
  delete S;
}

}  // extern "C"
