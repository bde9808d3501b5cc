// Continuous-batching server: many independent simulations on one GPU.
//
// Each simulation is an ordinary problem (its own sketch, Krylov basis and hierarchy, all in
// its own device arena) admitted when its arena fits the server's HBM budget; with
// queue_admission set, a simulation that does not fit yet waits (requests may already be
// queued for it) and is admitted, oldest first, as soon as closed simulations free enough of
// the budget. Requests (the surfaces and right-hand side of a simulation's next system) queue
// per simulation, first in first out. A tick takes the oldest request of idle simulations (at
// most one request each, up to a workgroup budget: the next simulation in round-robin order
// and those whose next solve is predicted to take at most twice as long) and runs them in one
// launch of the solve kernel: consecutive workgroup clusters, one per request, each running
// the same solve as sa_solve. Up to max_inflight ticks run at once, each on a stream of its
// own, so a long solve holds back only its own tick: as soon as any tick ends, its
// simulations' next requests and newly arrived ones form the next tick while the others keep
// running. A simulation is in at most one tick at a time, which keeps its solves in sequence.
//
// Co-residency of the clusters: every tick gets at most capacity / max_inflight workgroups
// (capacity = workgroups of the solve kernels the device holds at once), and a tick is only
// launched after the one it replaces has finished, so all workgroups of all running ticks fit
// on the device together and every cluster is resident as a whole. Ticks are therefore plain
// launches that run concurrently (cooperative launches would be serialised); the cluster
// barriers keep their bounded waits as a backstop: a cluster that times out flags its solve
// SA_EDEVICE, and the simulation's remaining requests complete with that status.
//
// Ordering: device inputs are read on the tick's stream after an event recorded on the
// server's stream at submit (the stream given at creation, on which the caller produces
// them). Every entry point takes the server's mutex, so submit and poll may be called from
// different host threads; a waiting poll releases it between checks.
#include <chrono>
#include <deque>
#include <mutex>
#include <thread>

#include "host.h"

using namespace sa;

namespace {

constexpr int MAX_INFLIGHT = 16;

double now_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
  uint64_t ticket = 0;
  const double *eta_p = nullptr, *eta_c = nullptr, *b = nullptr;  // device inputs
  std::vector<double> host;  // host inputs staged at submit: eta_p | eta_c | b
  hipEvent_t ready = nullptr;  // device inputs: recorded on the server's stream at submit
  double* x_out = nullptr;     // where the solution goes at completion (or null)
  int32_t x_mem = SA_MEM_HOST;
  double t_submit = 0.0;
};

struct Sim {
  bool open = false;     // the id is in use
  sa_problem* p = nullptr;  // null while waiting for admission
  int64_t bytes = 0;
  std::deque<Request> queue;
  int inflight = 0;       // requests in launched ticks not yet harvested
  int last_iters = 100;   // Arnoldi steps of its last solve (a guess before the first)
  bool failed = false;    // device error or failed admission: requests complete with `code`
  int code = SA_OK;
  // inputs of a simulation waiting for admission
  uint64_t wait_seq = 0;
  sa_grid grid{};
  std::vector<double> h;
  sa_options opt{};
};

// Predicted duration of a simulation's next solve, in arbitrary units: its last step count
// times the work per workgroup, floored where a step is bound by latency rather than bytes.
double predicted_cost(const Sim& m) {
  const double per_wg = (double)m.p->n / (double)m.p->G;
  return (m.last_iters + 2.0) * (per_wg > 4096.0 ? per_wg : 4096.0);
}

struct Entry {
  int sim;
  uint64_t ticket;
  double t_submit, t_launch;
  std::vector<double> host;  // kept alive until the tick is harvested
  double* x_out;
  int32_t x_mem;
};

struct Slot {
  hipStream_t stream = nullptr;  // the slot's own stream
  BatchItem* h_items = nullptr;  // pinned
  BatchItem* d_items = nullptr;
  sa_solve_info* h_rep = nullptr;  // pinned
  sa_solve_info* d_rep = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  uint64_t seq = 0;  // launch order
  std::vector<Entry> entries;
};

}  // namespace

struct sa_server {
  mutable std::mutex mu;
  hipStream_t stream = nullptr;
  int device = 0;
  sa_server_options opt{};
  int64_t used = 0;
  std::vector<Sim> sims;
  Slot slots[MAX_INFLIGHT];
  int capacity = 0;       // co-resident workgroups of the solve kernels at lds_set
  size_t lds_set = 0;
  int cus = 0;
  int rr = 0;
  uint64_t next_ticket = 1;
  uint64_t next_wait = 1;
  int64_t queued = 0, inflight = 0;
  int running = 0;        // busy slots
  uint64_t launches = 0;
  std::deque<sa_completion> ready;
  std::vector<hipEvent_t> event_pool;
  std::chrono::steady_clock::time_point t0;
  hipEvent_t ev0 = nullptr;
  double ev0_ms = 0.0;
  // statistics (sa_server_stats)
  double st_solves = 0.0, st_launch_ms = 0.0, st_tick_ms = 0.0;
  double st_device_failed = 0.0;  // solves that ended with SA_EDEVICE (a bounded wait gave up)
};

extern "C" void sa_server_default_options(sa_server_options* o) {
  memset(o, 0, sizeof *o);
  o->hbm_budget = 0;
  o->max_inflight = 4;
  o->max_batch = 0;
  o->unknowns_per_workgroup = 20000;
  o->queue_admission = 0;
}

static int set_lds(sa_server* s, size_t lds) {
  if (lds <= s->lds_set && s->capacity > 0) return SA_OK;
  int rc = sa_reserve_solve_lds(lds);
  if (rc != SA_OK) return rc;
  int per_cu = 0, per_cu32 = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sa_solve_fn(SA_FP64), BLOCK, lds));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu32, sa_solve_fn(SA_FP32_IR), BLOCK, lds));
  if (per_cu32 < per_cu) per_cu = per_cu32;
  if (per_cu < 1) return sa_fail(SA_EARG, "sa_server: %zu bytes of LDS per workgroup do not fit", lds);
  s->lds_set = lds;
  s->capacity = per_cu * s->cus;
  return SA_OK;
}

static void destroy_unlocked(sa_server* s);

extern "C" int sa_server_create(const sa_server_options* optin, void* hip_stream, sa_server** out) {
  if (!out) return sa_fail(SA_EARG, "sa_server_create: null argument");
  *out = nullptr;
  sa_server_options opt;
  if (optin) opt = *optin; else sa_server_default_options(&opt);
  if (opt.max_inflight < 1 || opt.max_inflight > MAX_INFLIGHT)
    return sa_fail(SA_EARG, "sa_server_create: max_inflight in [1, %d]", MAX_INFLIGHT);
  if (opt.max_batch < 0 || opt.unknowns_per_workgroup < 1 || opt.hbm_budget < 0 ||
      (opt.queue_admission != 0 && opt.queue_admission != 1))
    return sa_fail(SA_EARG, "sa_server_create: bad options");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return sa_fail(SA_ENOTBUILT, "sa_server_create: no HIP device");
  sa_server* s = new sa_server();
  s->opt = opt;
  s->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&s->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, s->device) != hipSuccess) {
    delete s;
    return sa_fail(SA_EDEVICE, "sa_server_create: hipGetDeviceProperties failed");
  }
  s->cus = prop.multiProcessorCount;
  if (opt.hbm_budget == 0) {
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) {
      delete s;
      return sa_fail(SA_EDEVICE, "sa_server_create: hipMemGetInfo failed");
    }
    s->opt.hbm_budget = (int64_t)(0.9 * (double)freeb);
  }
  int rc = set_lds(s, 64 * 1024);
  if (rc != SA_OK) { delete s; return rc; }
  const int maxitems = s->capacity;
  hipError_t e = hipSuccess;
  for (int i = 0; i < s->opt.max_inflight && e == hipSuccess; ++i) {  // the slots in use only
    Slot& sl = s->slots[i];
    e = hipHostMalloc((void**)&sl.h_items, sizeof(BatchItem) * maxitems, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_rep, sizeof(sa_solve_info) * maxitems, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_items, sizeof(BatchItem) * maxitems);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_rep, sizeof(sa_solve_info) * maxitems);
    if (e == hipSuccess) e = hipEventCreate(&sl.done);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
  }
  if (e == hipSuccess) e = hipEventCreate(&s->ev0);
  if (e == hipSuccess) {
    s->t0 = std::chrono::steady_clock::now();
    e = hipEventRecord(s->ev0, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->ev0);
    s->ev0_ms = now_ms(s->t0);
  }
  if (e != hipSuccess) {
    destroy_unlocked(s);
    return sa_fail(SA_EDEVICE, "sa_server_create: %s", hipGetErrorString(e));
  }
  *out = s;
  return SA_OK;
}

static void release_event(sa_server* s, Request& r) {
  if (r.ready) s->event_pool.push_back(r.ready);
  r.ready = nullptr;
}

static void destroy_unlocked(sa_server* s) {
  if (s->stream) (void)hipStreamSynchronize(s->stream); else (void)hipDeviceSynchronize();
  for (Slot& sl : s->slots)
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  for (Sim& m : s->sims) {
    for (Request& r : m.queue) release_event(s, r);
    if (m.p) sa_destroy(m.p);
  }
  for (Slot& sl : s->slots) {
    if (sl.h_items) (void)hipHostFree(sl.h_items);
    if (sl.h_rep) (void)hipHostFree(sl.h_rep);
    if (sl.d_items) (void)hipFree(sl.d_items);
    if (sl.d_rep) (void)hipFree(sl.d_rep);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (hipEvent_t ev : s->event_pool) (void)hipEventDestroy(ev);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
}

extern "C" void sa_server_destroy(sa_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    destroy_unlocked(s);
  }
  delete s;
}

static Sim* sim_of(sa_server* s, int32_t id) {
  if (id < 0 || id >= (int32_t)s->sims.size() || !s->sims[id].open) return nullptr;
  return &s->sims[id];
}

// every queued request of m completes with status `code` (device error or failed admission)
static void fail_queue(sa_server* s, int id, int code) {
  Sim& m = s->sims[id];
  const double t = now_ms(s->t0);
  while (!m.queue.empty()) {
    Request& r = m.queue.front();
    sa_completion c;
    memset(&c, 0, sizeof c);
    c.ticket = r.ticket;
    c.sim = id;
    c.info.status = code;
    c.t_submit_ms = r.t_submit;
    c.t_launch_ms = t;
    c.t_done_ms = t;
    release_event(s, r);
    s->ready.push_back(c);
    m.queue.pop_front();
    s->queued -= 1;
  }
}

// create the problem of a simulation that fits the budget now
static int admit(sa_server* s, int id) {
  Sim& m = s->sims[id];
  sa_problem* p = nullptr;
  int rc = sa_create(&m.grid, m.h.data(), &m.opt, (void*)s->stream, &p);
  if (rc < 0) return rc;
  rc = set_lds(s, p->lds_solve);
  if (rc == SA_OK && p->G > s->capacity / s->opt.max_inflight)
    rc = sa_fail(SA_EARG, "sa_server_open: cluster of %d workgroups too large for this device", p->G);
  if (rc != SA_OK) {
    sa_destroy(p);
    return rc;
  }
  m.p = p;
  m.bytes = (int64_t)p->arena_bytes;
  s->used += m.bytes;
  m.h.clear();
  m.h.shrink_to_fit();
  return SA_OK;
}

// admit waiting simulations in the order they asked, while the oldest one fits
static void admit_waiting(sa_server* s) {
  for (;;) {
    int best = -1;
    for (size_t i = 0; i < s->sims.size(); ++i) {
      const Sim& m = s->sims[i];
      if (m.open && !m.p && !m.failed && (best < 0 || m.wait_seq < s->sims[best].wait_seq)) best = (int)i;
    }
    if (best < 0 || s->used + s->sims[best].bytes > s->opt.hbm_budget) return;
    const int rc = admit(s, best);
    if (rc != SA_OK) {
      Sim& m = s->sims[best];
      m.failed = true;
      m.code = rc;
      fail_queue(s, best, rc);
    }
  }
}

extern "C" int sa_server_open(sa_server* s, const sa_grid* grid, const double* h, const sa_options* optin,
                              int32_t* sim) {
  if (!s || !grid || !h || !sim) return sa_fail(SA_EARG, "sa_server_open: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  sa_options opt;
  if (optin) opt = *optin; else sa_default_options(&opt);
  if (opt.decay != SA_DECAY_SOLVES)
    return sa_fail(SA_EARG, "sa_server_open: requests carry no time labels (SA_DECAY_SOLVES only)");
  const int budget = s->capacity / s->opt.max_inflight;
  if (opt.cluster <= 0) {
    const int ncol = grid->bc == SA_PERIODIC ? grid->nx - 1 : grid->nx + 2;
    const int64_t n = (int64_t)ncol * (grid->nz + 1);
    int64_t G = (n + s->opt.unknowns_per_workgroup - 1) / s->opt.unknowns_per_workgroup;
    if (G > budget) G = budget;
    opt.cluster = (int)(G < 1 ? 1 : (G > 16 ? 16 : G));
  }
  if (opt.cluster > budget)
    return sa_fail(SA_EARG, "sa_server_open: cluster of %d workgroups exceeds a tick's %d", opt.cluster, budget);
  opt.profile = 0;
  const int64_t bytes = sa_problem_bytes(grid, h, &opt);
  if (bytes < 0) return (int)bytes;
  if (bytes > s->opt.hbm_budget)
    return sa_fail(SA_EBUSY, "sa_server_open: %lld bytes needed, the budget is %lld", (long long)bytes,
                   (long long)s->opt.hbm_budget);
  const bool fits = s->used + bytes <= s->opt.hbm_budget;
  if (!fits && !s->opt.queue_admission)
    return sa_fail(SA_EBUSY, "sa_server_open: %lld bytes needed, %lld of %lld in use", (long long)bytes,
                   (long long)s->used, (long long)s->opt.hbm_budget);
  int id = -1;
  for (size_t i = 0; i < s->sims.size(); ++i)
    if (!s->sims[i].open) { id = (int)i; break; }
  if (id < 0) { id = (int)s->sims.size(); s->sims.emplace_back(); }
  Sim& m = s->sims[id];
  m = Sim();
  m.open = true;
  m.grid = *grid;
  m.opt = opt;
  m.bytes = bytes;
  const int nphys = grid->bc == SA_PERIODIC ? grid->nx - 1 : grid->nx;
  m.h.assign(h, h + nphys);
  m.wait_seq = s->next_wait++;
  // admit now unless older simulations are still waiting (admission is first come, first served)
  bool older_waiting = false;
  for (const Sim& o : s->sims)
    if (&o != &m && o.open && !o.p && !o.failed) older_waiting = true;
  if (fits && !older_waiting) {
    const int rc = admit(s, id);
    if (rc != SA_OK) {
      m = Sim();
      return rc;
    }
  }
  *sim = id;
  return SA_OK;
}

extern "C" int32_t sa_server_admitted(const sa_server* s, int32_t id) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  if (id < 0 || id >= (int32_t)s->sims.size() || !s->sims[id].open) return -1;
  const Sim& m = s->sims[id];
  if (m.failed && !m.p) return -1;
  return m.p ? 1 : 0;
}

extern "C" int sa_server_close(sa_server* s, int32_t id) {
  if (!s) return sa_fail(SA_EARG, "sa_server_close: null server");
  std::lock_guard<std::mutex> lk(s->mu);
  Sim* m = sim_of(s, id);
  if (!m) return sa_fail(SA_EARG, "sa_server_close: no simulation %d", id);
  if (m->inflight > 0 || (!m->queue.empty() && !m->failed))
    return sa_fail(SA_EBUSY, "sa_server_close: simulation %d has work", id);
  fail_queue(s, id, m->code);
  if (m->p) {
    sa_destroy(m->p);
    s->used -= m->bytes;
  }
  *m = Sim();
  admit_waiting(s);
  return SA_OK;
}

extern "C" int sa_server_submit(sa_server* s, int32_t id, const double* eta_prev, const double* eta_cur,
                                const double* b, int32_t mem, double* x_out, uint64_t* ticket) {
  if (!s || !eta_prev || !eta_cur || !b) return sa_fail(SA_EARG, "sa_server_submit: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  Sim* m = sim_of(s, id);
  if (!m) return sa_fail(SA_EARG, "sa_server_submit: no simulation %d", id);
  if (m->failed || (m->p && m->p->broken))
    return sa_fail(SA_EDEVICE, "sa_server_submit: simulation %d unusable after an error", id);
  Request r;
  r.t_submit = now_ms(s->t0);
  r.x_out = x_out;
  r.x_mem = mem;
  if (mem == SA_MEM_DEVICE) {
    r.eta_p = eta_prev; r.eta_c = eta_cur; r.b = b;
    if (!s->event_pool.empty()) {
      r.ready = s->event_pool.back();
      s->event_pool.pop_back();
    } else {
      HIPCHK(hipEventCreateWithFlags(&r.ready, hipEventDisableTiming));
    }
    const hipError_t e = hipEventRecord(r.ready, s->stream);
    if (e != hipSuccess) {
      release_event(s, r);
      return sa_fail(SA_EDEVICE, "sa_server_submit: %s", hipGetErrorString(e));
    }
  } else if (mem == SA_MEM_HOST) {
    const int np = m->grid.bc == SA_PERIODIC ? m->grid.nx - 1 : m->grid.nx;
    const int64_t n = (int64_t)(m->grid.bc == SA_PERIODIC ? m->grid.nx - 1 : m->grid.nx + 2) * (m->grid.nz + 1);
    r.host.resize((size_t)2 * np + n);
    for (int i = 0; i < np; ++i) {
      if (!isfinite(eta_prev[i]) || !isfinite(eta_cur[i])) return sa_fail(SA_EGEOM, "sa_server_submit: non-finite surface");
      r.host[i] = eta_prev[i];
      r.host[np + i] = eta_cur[i];
    }
    memcpy(r.host.data() + 2 * np, b, (size_t)n * 8);
  } else {
    return sa_fail(SA_EARG, "sa_server_submit: bad mem");
  }
  r.ticket = s->next_ticket++;
  if (ticket) *ticket = r.ticket;
  m->queue.push_back(std::move(r));
  s->queued += 1;
  return SA_OK;
}

// collect the reports of finished ticks (no waiting)
static int harvest(sa_server* s) {
  for (int si = 0; si < MAX_INFLIGHT; ++si) {
    Slot& sl = s->slots[si];
    if (!sl.busy) continue;
    hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    HIPCHK(q);
    float el = 0.0f;
    HIPCHK(hipEventElapsedTime(&el, s->ev0, sl.done));
    const double t_done = s->ev0_ms + el;
    for (size_t i = 0; i < sl.entries.size(); ++i) {
      const Entry& en = sl.entries[i];
      sa_completion c;
      memset(&c, 0, sizeof c);
      c.ticket = en.ticket;
      c.sim = en.sim;
      c.info = sl.h_rep[i];
      c.t_submit_ms = en.t_submit;
      c.t_launch_ms = en.t_launch;
      c.t_done_ms = t_done;
      Sim& m = s->sims[en.sim];
      m.inflight -= 1;
      m.last_iters = c.info.iters;
      if (en.x_out && c.info.status >= 0) {  // the simulation's solution, before its next tick
        HIPCHK(hipMemcpyAsync(en.x_out, m.p->hp.x, (size_t)m.p->n * 8,
                              en.x_mem == SA_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, sl.stream));
        HIPCHK(hipStreamSynchronize(sl.stream));
      }
      if (c.info.status == SA_EDEVICE) {
        s->st_device_failed += 1.0;
        m.p->broken = true;
        m.failed = true;
        m.code = SA_EDEVICE;
      }
      s->ready.push_back(c);
    }
    s->st_tick_ms += t_done - (sl.entries.empty() ? t_done : sl.entries[0].t_launch);
    s->inflight -= (int64_t)sl.entries.size();
    sl.entries.clear();
    sl.busy = false;
    s->running -= 1;
  }
  // a simulation whose solve failed on the device takes no more work: its queue completes
  for (size_t i = 0; i < s->sims.size(); ++i)
    if (s->sims[i].open && s->sims[i].failed && !s->sims[i].queue.empty()) fail_queue(s, (int)i, s->sims[i].code);
  return SA_OK;
}

// launch one tick from the queued requests into a free slot; *launched = number of solves.
// The tick's solves run in one launch per precision (FP64 group first, then FP32 refinement)
// on the slot's stream, together at most capacity / max_inflight workgroups.
static int launch_tick(sa_server* s, int* launched) {
  *launched = 0;
  if (s->queued == 0 || s->running >= s->opt.max_inflight) return SA_OK;
  int si = -1;
  for (int i = 0; i < s->opt.max_inflight; ++i)
    if (!s->slots[i].busy) { si = i; break; }
  if (si < 0) return SA_OK;
  const auto t_begin = std::chrono::steady_clock::now();
  Slot& sl = s->slots[si];
  const int nsim = (int)s->sims.size();
  const int maxb = s->opt.max_batch > 0 ? s->opt.max_batch : s->capacity;
  // workgroups per tick: an equal share of the co-resident capacity per running tick (every
  // open simulation's cluster fits it)
  const int budget = s->capacity / s->opt.max_inflight;
  // pick the requests, at most one per idle simulation: the first idle simulation with work
  // from s->rr in round-robin order, then, scanning on, those whose next solve is predicted to
  // take at most twice as long as the first one's (a tick lasts as long as its slowest solve,
  // and every simulation is first within nsim ticks, so none is held back for good)
  std::vector<int> picked[2];
  int blocks[2] = {0, 0};
  int total = 0, first_id = -1;
  double limit = 0.0;
  for (int scanned = 0; scanned < nsim && total < maxb; ++scanned) {
    const int id = (s->rr + scanned) % nsim;
    Sim& m = s->sims[id];
    if (!m.open || !m.p || m.failed || m.queue.empty() || m.p->broken || m.inflight > 0) continue;
    if (first_id >= 0 && predicted_cost(m) > limit) continue;
    if (blocks[0] + blocks[1] + m.p->G > budget) {
      if (first_id < 0) break;
      continue;
    }
    const int g = m.p->opt.precision == SA_FP32_IR ? 1 : 0;
    blocks[g] += m.p->G;
    picked[g].push_back(id);
    ++total;
    if (first_id < 0) {
      first_id = id;
      limit = 2.0 * predicted_cost(m);
    }
  }
  s->rr = ((first_id >= 0 ? first_id : s->rr) + 1) % (nsim > 0 ? nsim : 1);
  if (total == 0) return SA_OK;
  const double t_launch = now_ms(s->t0);
  int nitems = 0;
  int start[2] = {0, 0}, count[2] = {0, 0};

  for (int g = 0; g < 2; ++g) {
    start[g] = nitems;
    int first = 0;
    for (int id : picked[g]) {
      Sim& m = s->sims[id];
      sa_problem* p = m.p;
      Request& r = m.queue.front();
      if (r.ready) {  // device inputs: after the caller's stream has produced them
        HIPCHK(hipStreamWaitEvent(sl.stream, r.ready, 0));
        release_event(s, r);
      }
      if (!r.host.empty()) {
        const int np = p->nphys;
        HIPCHK(hipMemcpyAsync(p->eta_own, r.host.data(), (size_t)2 * np * 8, hipMemcpyHostToDevice, sl.stream));
        HIPCHK(hipMemcpyAsync(p->b_own, r.host.data() + 2 * np, (size_t)p->n * 8, hipMemcpyHostToDevice, sl.stream));
        p->eta_p = p->eta_own;
        p->eta_c = p->eta_own + np;
        p->b = p->b_own;
      } else {
        p->eta_p = r.eta_p;
        p->eta_c = r.eta_c;
        p->b = r.b;
      }
      bool ewma = false;
      SolveArgs a = sa_prepare_solve(p, &ewma);
      a.out = (decltype(a.out))(sl.d_rep + nitems);
      BatchItem& it = sl.h_items[nitems];
      it.P = (decltype(it.P))p->dp;
      it.first = first;
      it.sketch = ewma ? 1 : 0;
      it.a = a;
      sa_commit_solve(p, a);
      first += p->G;
      sl.entries.push_back(Entry{id, r.ticket, r.t_submit, t_launch, std::move(r.host), r.x_out, r.x_mem});
      m.queue.pop_front();
      m.inflight += 1;
      s->queued -= 1;
      ++nitems;
    }
    count[g] = nitems - start[g];
  }
  HIPCHK(hipMemcpyAsync(sl.d_items, sl.h_items, sizeof(BatchItem) * nitems, hipMemcpyHostToDevice, sl.stream));
  BatchItem unused;
  memset(&unused, 0, sizeof unused);
  for (int g = 0; g < 2; ++g) {
    if (!count[g]) continue;
    const BatchItem* items = sl.d_items + start[g];
    int ni = count[g];
    void* args[] = {(void*)&items, (void*)&ni, (void*)&unused};
    const void* fn = sa_solve_fn(g ? SA_FP32_IR : SA_FP64);
    HIPCHK(hipLaunchKernel(fn, dim3(blocks[g]), dim3(BLOCK), args, s->lds_set, sl.stream));
  }
  HIPCHK(hipMemcpyAsync(sl.h_rep, sl.d_rep, sizeof(sa_solve_info) * nitems, hipMemcpyDeviceToHost, sl.stream));
  HIPCHK(hipEventRecord(sl.done, sl.stream));
  sl.busy = true;
  sl.seq = ++s->launches;
  s->running += 1;
  s->inflight += nitems;
  s->st_solves += nitems;
  s->st_launch_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
  *launched = nitems;
  return SA_OK;
}

// harvest, admit, launch as many ticks as there are free slots and queued requests
static int progress(sa_server* s) {
  int rc = harvest(s);
  if (rc) return rc;
  admit_waiting(s);
  for (;;) {
    int launched = 0;
    rc = launch_tick(s, &launched);
    if (rc) return rc;
    if (!launched) return SA_OK;
  }
}

extern "C" int sa_server_poll(sa_server* s, sa_completion* out, int32_t max, int32_t* n_out, int32_t wait_us) {
  if (!s || !n_out || (max > 0 && !out)) return sa_fail(SA_EARG, "sa_server_poll: bad arguments");
  *n_out = 0;
  const auto t_begin = std::chrono::steady_clock::now();
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    const int rc = progress(s);
    if (rc) return rc;
    const bool waited_enough =
        wait_us == 0 ||
        (wait_us > 0 && std::chrono::steady_clock::now() - t_begin >= std::chrono::microseconds(wait_us));
    // nothing will complete while no tick runs (the queues are launched by progress above)
    if (!s->ready.empty() || waited_enough || s->running == 0) break;
    lk.unlock();
    std::this_thread::sleep_for(std::chrono::microseconds(20));
    lk.lock();
  }
  int32_t cnt = 0;
  while (cnt < max && !s->ready.empty()) {
    out[cnt++] = s->ready.front();
    s->ready.pop_front();
  }
  *n_out = cnt;
  return SA_OK;
}

extern "C" int64_t sa_server_outstanding(const sa_server* s) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  return s->queued + s->inflight + (int64_t)s->ready.size();
}

extern "C" int64_t sa_server_bytes_used(const sa_server* s) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  return s->used;
}

extern "C" double sa_server_clock_ms(const sa_server* s) { return s ? now_ms(s->t0) : -1.0; }

extern "C" int sa_server_stats(const sa_server* s, double* out, int32_t n) {
  if (!s || !out || n < 1) return sa_fail(SA_EARG, "sa_server_stats: bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  const double v[7] = {(double)s->launches, s->st_solves,     s->st_launch_ms,
                       s->st_tick_ms,       (double)s->capacity, (double)(s->capacity / s->opt.max_inflight),
                       s->st_device_failed};
  for (int i = 0; i < n && i < 7; ++i) out[i] = v[i];
  return SA_OK;
}

extern "C" sa_problem* sa_server_problem(sa_server* s, int32_t id) {
  if (!s) return nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  Sim* m = sim_of(s, id);
  // its device state may only be read once its last tick has been harvested
  return (m && m->p && m->inflight == 0) ? m->p : nullptr;
}
