// Continuous-batching server: many independent simulations on one GPU.
//
// Each simulation is an ordinary problem (its own sketch, Krylov basis and hierarchy, all in
// its own device arena) admitted when its arena fits the server's HBM budget. Requests (the
// surfaces and right-hand side of a simulation's next system) queue per simulation, first in
// first out. A tick takes the oldest request of idle simulations (at most one request each, up
// to a workgroup budget: the next simulation in round-robin order and those whose next solve
// is predicted to take at most twice as long) and runs them in one launch of the solve kernel:
// consecutive workgroup clusters, one per request, each running the same solve as sa_solve.
// Up to max_inflight ticks run at once, each on a stream of its own, so a long solve holds
// back only its own tick: as soon as any tick ends, its simulations' next requests and newly
// arrived ones form the next tick while the others keep running. A simulation is in at most
// one tick at a time, which keeps its solves in sequence.
//
// Co-residency of the clusters: every tick gets at most capacity / max_inflight workgroups
// (capacity = workgroups of the solve kernels the device holds at once), and a tick is only
// launched after the one it replaces has finished, so all workgroups of all running ticks fit
// on the device together and every cluster is resident as a whole. Ticks are therefore plain
// launches that run concurrently (cooperative launches would be serialised); the cluster
// barriers keep their bounded waits as a backstop.
#include <chrono>
#include <deque>

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
  double t_submit = 0.0;
};

struct Sim {
  sa_problem* p = nullptr;
  int64_t bytes = 0;
  std::deque<Request> queue;
  int inflight = 0;    // requests in launched ticks not yet harvested
  int last_iters = 100;  // Arnoldi steps of its last solve (a guess before the first)
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
  int64_t queued = 0, inflight = 0;
  int running = 0;        // busy slots
  uint64_t launches = 0;
  std::deque<sa_completion> ready;
  std::chrono::steady_clock::time_point t0;
  hipEvent_t ev0 = nullptr;
  double ev0_ms = 0.0;
};

extern "C" void sa_server_default_options(sa_server_options* o) {
  memset(o, 0, sizeof *o);
  o->hbm_budget = 0;
  o->max_inflight = 4;
  o->max_batch = 0;
  o->unknowns_per_workgroup = 20000;
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

extern "C" int sa_server_create(const sa_server_options* optin, void* hip_stream, sa_server** out) {
  if (!out) return sa_fail(SA_EARG, "sa_server_create: null argument");
  *out = nullptr;
  sa_server_options opt;
  if (optin) opt = *optin; else sa_server_default_options(&opt);
  if (opt.max_inflight < 1 || opt.max_inflight > MAX_INFLIGHT)
    return sa_fail(SA_EARG, "sa_server_create: max_inflight in [1, %d]", MAX_INFLIGHT);
  if (opt.max_batch < 0 || opt.unknowns_per_workgroup < 1 || opt.hbm_budget < 0)
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
    sa_server_destroy(s);
    return sa_fail(SA_EDEVICE, "sa_server_create: %s", hipGetErrorString(e));
  }
  *out = s;
  return SA_OK;
}

extern "C" void sa_server_destroy(sa_server* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream); else (void)hipDeviceSynchronize();
  for (Slot& sl : s->slots)
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  for (Sim& m : s->sims)
    if (m.p) sa_destroy(m.p);
  for (Slot& sl : s->slots) {
    if (sl.h_items) (void)hipHostFree(sl.h_items);
    if (sl.h_rep) (void)hipHostFree(sl.h_rep);
    if (sl.d_items) (void)hipFree(sl.d_items);
    if (sl.d_rep) (void)hipFree(sl.d_rep);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  delete s;
}

extern "C" int sa_server_open(sa_server* s, const sa_grid* grid, const double* h, const sa_options* optin,
                              int32_t* sim) {
  if (!s || !grid || !h || !sim) return sa_fail(SA_EARG, "sa_server_open: null argument");
  sa_options opt;
  if (optin) opt = *optin; else sa_default_options(&opt);
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
  if (s->used + bytes > s->opt.hbm_budget)
    return sa_fail(SA_EBUSY, "sa_server_open: %lld bytes needed, %lld of %lld in use", (long long)bytes,
                   (long long)s->used, (long long)s->opt.hbm_budget);
  sa_problem* p = nullptr;
  int rc = sa_create(grid, h, &opt, (void*)s->stream, &p);
  if (rc < 0) return rc;
  rc = set_lds(s, p->lds_solve);
  if (rc == SA_OK && p->G > s->capacity / s->opt.max_inflight)
    rc = sa_fail(SA_EARG, "sa_server_open: cluster of %d workgroups too large for this device", p->G);
  if (rc != SA_OK) {
    sa_destroy(p);
    return rc;
  }
  int id = -1;
  for (size_t i = 0; i < s->sims.size(); ++i)
    if (!s->sims[i].p) { id = (int)i; break; }
  if (id < 0) { id = (int)s->sims.size(); s->sims.emplace_back(); }
  s->sims[id].p = p;
  s->sims[id].bytes = p->arena_bytes;
  s->used += (int64_t)p->arena_bytes;
  *sim = id;
  return SA_OK;
}

static Sim* sim_of(sa_server* s, int32_t id) {
  if (id < 0 || id >= (int32_t)s->sims.size() || !s->sims[id].p) return nullptr;
  return &s->sims[id];
}

extern "C" int sa_server_close(sa_server* s, int32_t id) {
  if (!s) return sa_fail(SA_EARG, "sa_server_close: null server");
  Sim* m = sim_of(s, id);
  if (!m) return sa_fail(SA_EARG, "sa_server_close: no simulation %d", id);
  if (!m->queue.empty() || m->inflight > 0) return sa_fail(SA_EBUSY, "sa_server_close: simulation %d has work", id);
  sa_destroy(m->p);
  s->used -= m->bytes;
  *m = Sim();
  return SA_OK;
}

extern "C" int sa_server_submit(sa_server* s, int32_t id, const double* eta_prev, const double* eta_cur,
                                const double* b, int32_t mem, uint64_t* ticket) {
  if (!s || !eta_prev || !eta_cur || !b) return sa_fail(SA_EARG, "sa_server_submit: null argument");
  Sim* m = sim_of(s, id);
  if (!m) return sa_fail(SA_EARG, "sa_server_submit: no simulation %d", id);
  if (m->p->broken) return sa_fail(SA_EDEVICE, "sa_server_submit: simulation %d unusable after a device error", id);
  Request r;
  r.ticket = s->next_ticket++;
  r.t_submit = now_ms(s->t0);
  if (mem == SA_MEM_DEVICE) {
    r.eta_p = eta_prev; r.eta_c = eta_cur; r.b = b;
  } else if (mem == SA_MEM_HOST) {
    const int np = m->p->nphys, n = m->p->n;
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
  if (ticket) *ticket = r.ticket;
  m->queue.push_back(std::move(r));
  s->queued += 1;
  return SA_OK;
}

// collect the reports of finished ticks; with `wait`, block on the oldest running tick first
static int harvest(sa_server* s, bool wait) {
  if (wait) {
    int oldest = -1;
    for (int i = 0; i < MAX_INFLIGHT; ++i)
      if (s->slots[i].busy && (oldest < 0 || s->slots[i].seq < s->slots[oldest].seq)) oldest = i;
    if (oldest >= 0) HIPCHK(hipEventSynchronize(s->slots[oldest].done));
  }
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
      if (c.info.status == SA_EDEVICE) m.p->broken = true;
      s->ready.push_back(c);
    }
    s->inflight -= (int64_t)sl.entries.size();
    sl.entries.clear();
    sl.busy = false;
    s->running -= 1;
  }
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
    if (!m.p || m.queue.empty() || m.p->broken || m.inflight > 0) continue;
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
      sl.entries.push_back(Entry{id, r.ticket, r.t_submit, t_launch, std::move(r.host)});
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
  *launched = nitems;
  return SA_OK;
}

extern "C" int sa_server_poll(sa_server* s, sa_completion* out, int32_t max, int32_t* n_out, int32_t wait) {
  if (!s || !n_out || (max > 0 && !out)) return sa_fail(SA_EARG, "sa_server_poll: bad arguments");
  *n_out = 0;
  int rc = harvest(s, false);
  if (rc) return rc;
  for (;;) {
    int launched = 0;
    rc = launch_tick(s, &launched);
    if (rc) return rc;
    if (!launched) break;
  }
  if (wait && s->ready.empty() && s->running > 0) {
    rc = harvest(s, true);
    if (rc) return rc;
    for (;;) {  // refill the slot that just freed
      int launched = 0;
      rc = launch_tick(s, &launched);
      if (rc) return rc;
      if (!launched) break;
    }
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
  return s ? s->queued + s->inflight + (int64_t)s->ready.size() : -1;
}

extern "C" int64_t sa_server_bytes_used(const sa_server* s) { return s ? s->used : -1; }

extern "C" sa_problem* sa_server_problem(sa_server* s, int32_t id) {
  if (!s) return nullptr;
  Sim* m = sim_of(s, id);
  // its device state may only be read once its last tick has been harvested
  return (m && m->inflight == 0) ? m->p : nullptr;
}
