// Serving loop: continuous batching of independent Poisson solves.
//
// A persistent worker thread drives up to 16 caller-owned HIP streams
// ("slots").  Requests (stream id, grid size, density, output array) queue in
// arrival order and are admitted while a slot is free and their device
// footprint -- plan workspace plus the stream's cached potential -- fits the
// caller's device arena (least recently used idle plans and cached potentials
// are released to make room).  Plan workspaces and cached potentials are
// ranges of that one arena, handed out first-fit from a free list whose
// released ranges merge with their neighbours; the server itself allocates no
// device memory and creates no stream.  Each admitted request first waits on
// its slot for the work the caller had queued on its own stream before
// submitting, then advances one multigrid iteration at a time (a graph launch
// of the plan's captured step), so requests of different sizes overlap on the
// device; the worker polls one event per slot and never blocks on the device.
// When a request converges its potential is written to the caller's array
// and kept in the arena as the next initial guess of the same stream id
// (Section 2.1: the previous potential as initial estimate).  Results do not
// depend on the mix: every plan of a size computes identically and all
// reductions run in a fixed order.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "plan_impl.h"

using namespace psn;

namespace {

constexpr int kMaxSlots = 16;
constexpr size_t kAlign = 256;

size_t round_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// First-fit ranges of the caller's device arena.  free_ maps the offset of
// every free range to its size; adjacent free ranges are always merged.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  std::atomic<size_t> used{0};
  std::map<size_t, size_t> free_;

  void init(void* b, size_t bytes) {
    base = (char*)b;
    cap = bytes & ~(kAlign - 1);
    free_.clear();
    if (cap) free_[0] = cap;
    used = 0;
  }
  void* take(size_t bytes) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used += bytes;
        return base + off;
      }
    return nullptr;
  }
  void give(void* p, size_t bytes) {
    if (!p) return;
    bytes = round_up(bytes);
    size_t off = (size_t)((char*)p - base);
    used -= bytes;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {  // merge with the next range
      bytes += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {  // and with the previous one
        pv->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  // would first-fit placement of every size, in order, succeed now?
  bool fits(const std::vector<size_t>& sizes) const {
    std::vector<size_t> room;
    for (auto& kv : free_) room.push_back(kv.second);
    for (size_t b : sizes) {
      b = round_up(b);
      bool ok = false;
      for (size_t& r : room)
        if (r >= b) {
          r -= b;
          ok = true;
          break;
        }
      if (!ok) return false;
    }
    return true;
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct PlanEntry {
  poisson_plan_t plan = nullptr;
  void* ws = nullptr;
  size_t bytes = 0;
  int n = 0;
  bool busy = false;
  uint64_t last_use = 0;
};

struct CacheEntry {
  double* phi = nullptr;
  size_t bytes = 0;
  int n = 0;
  bool in_use = false;
  bool valid = false;
  uint64_t last_use = 0;
};

enum Phase { kQueued = 0, kSetup, kStep, kFinishing, kDone };

struct Request {
  int64_t ticket = 0;
  int32_t stream_id = 0;
  int32_t n = 0;
  const double* rho = nullptr;
  double* phi = nullptr;
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  int phase = kQueued;
  int status = 0;
  int iterations = 0;
  bool warm = false;
  double bnorm = 0.0, rel = 0.0;
  int slot = -1;
  PlanEntry* plan = nullptr;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
};

}  // namespace

struct poisson_server_s {
  size_t budget = 0;
  int max_slots = 1;
  bool mixed = true, warm = true, graphs = true;
  int lmax = 8, nu = 2, max_iter = 100;
  double tol = 1e-8;
  int device = 0;
  Arena arena;                          // the caller's device memory
  hipStream_t streams[kMaxSlots] = {};  // the caller's slot streams
  hipEvent_t events[kMaxSlots] = {};
  Request* slot_req[kMaxSlots] = {};
  double* pinned = nullptr;  // 2 doubles per slot
  std::vector<PlanEntry*> plans;
  std::unordered_map<int, CacheEntry> cache;
  std::unordered_map<int, int> running;  // stream id -> running requests (0 or 1)
  uint64_t clock = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::unordered_map<int64_t, Request*> reqs;
  int64_t next_ticket = 1;
  int active = 0;
  std::deque<std::pair<int, int>> reserve;  // (n, count) requests for the worker
  int reserve_pending = 0;
  int reserve_status = 0;
  std::atomic<bool> stop{false};
  std::thread worker;
  int fatal = 0;
};

namespace {

poisson_grid_t grid_for(int n) {
  poisson_grid_t g;
  memset(&g, 0, sizeof g);
  g.coord = POISSON_CARTESIAN;
  g.n[0] = g.n[1] = g.n[2] = n;
  g.lo[0] = g.lo[1] = g.lo[2] = 0.0;
  g.hi[0] = g.hi[1] = g.hi[2] = 1.0;
  g.ghost = 1;
  g.pitch[0] = n + 1;
  g.pitch[1] = (int64_t)(n + 1) * (n + 1);
  return g;
}

poisson_opts_t opts_for(const poisson_server_s* S) {
  poisson_opts_t o;
  poisson_default_opts(&o, S->mixed ? POISSON_MG_IR32 : POISSON_MG);
  o.lmax = S->lmax;
  o.nu1 = o.nu2 = S->nu;
  o.max_iter = S->max_iter;
  return o;
}

size_t plan_bytes(const poisson_server_s* S, int n) {
  poisson_grid_t g = grid_for(n);
  poisson_opts_t o = opts_for(S);
  return poisson_workspace_bytes(&g, &o);
}

size_t phi_bytes(int n) { return sizeof(double) * (size_t)(n + 1) * (n + 1) * (n + 1); }

// Arena ranges a request still needs to start now.
std::vector<size_t> need_ranges(poisson_server_s* S, const Request* r) {
  std::vector<size_t> need;
  bool have_plan = false;
  for (PlanEntry* p : S->plans)
    if (!p->busy && p->n == r->n) have_plan = true;
  if (!have_plan) need.push_back(plan_bytes(S, r->n));
  if (S->warm) {
    auto it = S->cache.find(r->stream_id);
    if (it == S->cache.end() || it->second.n != r->n) need.push_back(phi_bytes(r->n));
  }
  return need;
}

// Release idle plans and cached potentials (least recently used first) until
// ranges of the sizes in `need` can be taken from the arena, sparing plans of
// size keep_n (about to be reused) and the cached potential of keep_stream.
// Returns true when they fit.
bool make_room(poisson_server_s* S, const std::vector<size_t>& need, int keep_stream, int keep_n) {
  while (!S->arena.fits(need)) {
    uint64_t best = UINT64_MAX;
    int kind = -1;
    size_t pi = 0;
    int ck = 0;
    int idle_keep = 0;  // one idle plan of size keep_n is always spared
    for (PlanEntry* p : S->plans)
      if (!p->busy && p->n == keep_n) ++idle_keep;
    for (size_t i = 0; i < S->plans.size(); ++i)
      if (!S->plans[i]->busy && (S->plans[i]->n != keep_n || idle_keep > 1) && S->plans[i]->last_use < best) {
        best = S->plans[i]->last_use;
        kind = 0;
        pi = i;
      }
    // a stream's cached potential of another size is replaced anyway
    for (auto& kv : S->cache)
      if (!kv.second.in_use && (kv.first != keep_stream || kv.second.n != keep_n) && kv.second.last_use < best) {
        best = kv.second.last_use;
        kind = 1;
        ck = kv.first;
      }
    if (kind < 0) return false;
    if (kind == 0) {
      PlanEntry* p = S->plans[pi];
      poisson_plan_destroy(p->plan);
      S->arena.give(p->ws, p->bytes);
      delete p;
      S->plans.erase(S->plans.begin() + pi);
    } else {
      CacheEntry& c = S->cache[ck];
      S->arena.give(c.phi, c.bytes);
      S->cache.erase(ck);
    }
  }
  return true;
}

PlanEntry* take_plan(poisson_server_s* S, int n, int slot, int* status, bool force_new = false) {
  PlanEntry* pe = nullptr;
  for (PlanEntry* p : S->plans)
    if (!force_new && !p->busy && p->n == n) {
      pe = p;
      break;
    }
  if (!pe) {
    pe = new PlanEntry();
    pe->n = n;
    pe->bytes = plan_bytes(S, n);
    pe->ws = S->arena.take(pe->bytes);
    if (!pe->ws) {
      set_error("no arena range of %zu bytes for a plan", pe->bytes);
      delete pe;
      *status = POISSON_EADMIT;
      return nullptr;
    }
    poisson_grid_t g = grid_for(n);
    poisson_opts_t o = opts_for(S);
    int s = poisson_plan(&pe->plan, &g, &o, pe->ws, pe->bytes, S->streams[slot]);
    if (s != POISSON_OK) {
      S->arena.give(pe->ws, pe->bytes);
      delete pe;
      *status = s;
      return nullptr;
    }
    if (S->graphs && cart_prepare_graph(pe->plan) != POISSON_OK) {
      poisson_plan_destroy(pe->plan);
      S->arena.give(pe->ws, pe->bytes);
      delete pe;
      *status = POISSON_EHIP;
      return nullptr;
    }
    S->plans.push_back(pe);
  }
  pe->busy = true;
  pe->last_use = ++S->clock;
  pe->plan->st = S->streams[slot];
  return pe;
}

void complete(poisson_server_s* S, Request* r, int status) {
  const int slot = r->slot;
  if (r->plan) {
    r->plan->busy = false;
    r->plan = nullptr;
  }
  auto it = S->cache.find(r->stream_id);
  if (it != S->cache.end()) it->second.in_use = false;
  S->running.erase(r->stream_id);
  if (r->ready) {
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  r->status = status;
  r->t_done = now_ms();
  r->phase = kDone;
  if (slot >= 0) S->slot_req[slot] = nullptr;
  r->slot = -1;
  --S->active;
  S->cv.notify_all();
}

int fail_hip(poisson_server_s* S, Request* r) {
  complete(S, r, POISSON_EHIP);
  return POISSON_EHIP;
}

// Enqueue the solve setup of an admitted request on its slot.
void start(poisson_server_s* S, Request* r, int slot) {
  r->slot = slot;
  r->t_start = now_ms();
  S->slot_req[slot] = r;
  hipStream_t st = S->streams[slot];
  int status = 0;
  r->plan = take_plan(S, r->n, slot, &status);
  if (!r->plan) {
    complete(S, r, status);
    return;
  }
  // the caller's work on rho and phi queued before submission comes first
  if (r->ready && hipStreamWaitEvent(st, r->ready, 0) != hipSuccess) {
    fail_hip(S, r);
    return;
  }
  const size_t pb = phi_bytes(r->n);
  r->warm = false;
  if (S->warm) {
    CacheEntry& c = S->cache[r->stream_id];
    if (c.phi && c.n != r->n) {
      S->arena.give(c.phi, c.bytes);
      c = CacheEntry();
    }
    if (!c.phi) {
      c.phi = (double*)S->arena.take(pb);
      if (!c.phi) {
        set_error("no arena range of %zu bytes for a cached potential", pb);
        complete(S, r, POISSON_EADMIT);
        return;
      }
      c.bytes = pb;
      c.n = r->n;
    }
    c.in_use = true;
    c.last_use = ++S->clock;
    r->warm = c.valid;
  }
  hipError_t e = r->warm ? hipMemcpyAsync(r->phi, S->cache[r->stream_id].phi, pb, hipMemcpyDeviceToDevice, st)
                         : hipMemsetAsync(r->phi, 0, pb, st);
  if (e != hipSuccess) {
    fail_hip(S, r);
    return;
  }
  poisson_plan_t P = r->plan->plan;
  if (cart_setup(P, r->rho, r->phi) != POISSON_OK ||
      hipMemcpyAsync(S->pinned + 2 * slot, &P->scal->v[kBnorm2], 2 * sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipEventRecord(S->events[slot], st) != hipSuccess) {
    fail_hip(S, r);
    return;
  }
  r->phase = kSetup;
}

// Handle a slot whose last enqueued work has finished.
void advance(poisson_server_s* S, Request* r) {
  const int slot = r->slot;
  hipStream_t st = S->streams[slot];
  poisson_plan_t P = r->plan->plan;
  if (r->phase == kFinishing) {
    if (S->warm) S->cache[r->stream_id].valid = true;
    complete(S, r, r->rel <= S->tol ? POISSON_OK : POISSON_WARN_MAXITER);
    return;
  }
  if (r->phase == kSetup) r->bnorm = sqrt(std::max(S->pinned[2 * slot], 0.0));
  const double rr = sqrt(std::max(S->pinned[2 * slot + 1], 0.0));
  r->rel = r->bnorm > 0.0 ? rr / r->bnorm : rr;
  if (!isfinite(r->rel)) {
    complete(S, r, POISSON_ENUMERIC);
    return;
  }
  if (r->rel <= S->tol || r->iterations >= S->max_iter) {
    if (cart_finish(P, r->phi) != POISSON_OK) {
      fail_hip(S, r);
      return;
    }
    if (S->warm &&
        hipMemcpyAsync(S->cache[r->stream_id].phi, r->phi, phi_bytes(r->n), hipMemcpyDeviceToDevice, st) != hipSuccess) {
      fail_hip(S, r);
      return;
    }
    if (hipEventRecord(S->events[slot], st) != hipSuccess) {
      fail_hip(S, r);
      return;
    }
    r->phase = kFinishing;
    return;
  }
  if (cart_step(P, S->graphs) != POISSON_OK ||
      hipMemcpyAsync(S->pinned + 2 * slot + 1, &P->scal->v[kRes2], sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipEventRecord(S->events[slot], st) != hipSuccess) {
    fail_hip(S, r);
    return;
  }
  ++r->iterations;
  r->phase = kStep;
}

// Create idle plans (and their graphs) ahead of traffic so that no request
// pays for plan construction; runs on the worker thread.
void do_reserve(poisson_server_s* S, int n, int count) {
  int have = 0;
  for (PlanEntry* p : S->plans)
    if (p->n == n) ++have;
  int status = POISSON_OK;
  for (; have < count && status == POISSON_OK; ++have) {
    if (!make_room(S, {plan_bytes(S, n)}, -1, n)) {
      status = POISSON_EADMIT;
      break;
    }
    PlanEntry* pe = take_plan(S, n, 0, &status, true);
    if (pe) pe->busy = false;
  }
  (void)hipStreamSynchronize(S->streams[0]);
  std::lock_guard<std::mutex> lk(S->mu);
  if (status != POISSON_OK) S->reserve_status = status;
  --S->reserve_pending;
  S->cv.notify_all();
}

void worker_loop(poisson_server_s* S) {
  (void)hipSetDevice(S->device);
  while (!S->stop.load()) {
    bool progress = false;
    while (true) {
      std::pair<int, int> job;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->reserve.empty()) break;
        job = S->reserve.front();
        S->reserve.pop_front();
      }
      do_reserve(S, job.first, job.second);
      progress = true;
    }
    // admission in arrival order; a stream's next request waits for the
    // previous one, whose potential is its initial guess
    while (true) {
      Request* r = nullptr;
      int slot = -1;
      size_t qi = 0;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        for (int i = 0; i < S->max_slots; ++i)
          if (!S->slot_req[i]) {
            slot = i;
            break;
          }
        if (slot < 0) break;
        for (qi = 0; qi < S->queue.size(); ++qi)
          if (!S->running.count(S->queue[qi]->stream_id)) {
            r = S->queue[qi];
            break;
          }
        if (!r) break;
      }
      if (!make_room(S, need_ranges(S, r), r->stream_id, r->n)) {
        if (S->active == 0) {  // nothing will free up: the request can never fit
          std::lock_guard<std::mutex> lk(S->mu);
          S->queue.erase(S->queue.begin() + qi);
          if (r->ready) {
            (void)hipEventDestroy(r->ready);
            r->ready = nullptr;
          }
          r->phase = kDone;
          r->status = POISSON_EADMIT;
          r->t_done = now_ms();
          S->cv.notify_all();
          continue;
        }
        break;  // wait for a running request to retire
      }
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->queue.erase(S->queue.begin() + qi);
        ++S->active;
      }
      S->running[r->stream_id] = 1;
      start(S, r, slot);
      progress = true;
    }
    // advance every slot whose work has completed
    for (int i = 0; i < S->max_slots; ++i) {
      Request* r = S->slot_req[i];
      if (!r) continue;
      const hipError_t q = hipEventQuery(S->events[i]);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        fail_hip(S, r);
        continue;
      }
      advance(S, r);
      progress = true;
    }
    if (!progress) {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->active == 0 && S->queue.empty() && S->reserve.empty())
        S->cv.wait_for(lk, std::chrono::milliseconds(50));
      else
        std::this_thread::yield();
    }
  }
}

}  // namespace

extern "C" {

int poisson_server_create(poisson_server_t* out, void* d_arena, size_t arena_bytes, int32_t max_slots,
                          void* const* slot_streams, int32_t mixed, int32_t lmax, int32_t nu, double tol,
                          int32_t warm_start, int32_t use_graphs) {
  if (!out || !d_arena || !slot_streams || max_slots < 1 || max_slots > kMaxSlots || lmax < -1 ||
      lmax > kLmaxMax || nu < 1 || !(tol > 0.0)) {
    set_error("invalid server option");
    return POISSON_EINVAL;
  }
  if (((uintptr_t)d_arena & (kAlign - 1)) != 0) {
    set_error("the arena must be %zu-byte aligned", kAlign);
    return POISSON_EWORKSPACE;
  }
  for (int i = 0; i < max_slots; ++i)
    if (!slot_streams[i]) {
      set_error("slot stream %d is the NULL stream", i);
      return POISSON_EINVAL;
    }
  poisson_server_s* S = new poisson_server_s();
  S->budget = arena_bytes & ~(kAlign - 1);
  S->arena.init(d_arena, arena_bytes);
  S->max_slots = max_slots;
  S->mixed = mixed != 0;
  S->lmax = lmax;
  S->nu = nu;
  S->tol = tol;
  S->warm = warm_start != 0;
  S->graphs = use_graphs != 0;
  if (hipGetDevice(&S->device) != hipSuccess || hipHostMalloc((void**)&S->pinned, 2 * kMaxSlots * sizeof(double),
                                                               hipHostMallocDefault) != hipSuccess) {
    set_error("server set-up failed");
    delete S;
    return POISSON_EHIP;
  }
  for (int i = 0; i < max_slots; ++i) {
    S->streams[i] = (hipStream_t)slot_streams[i];
    if (hipEventCreateWithFlags(&S->events[i], hipEventDisableTiming) != hipSuccess) {
      set_error("server event creation failed");
      poisson_server_destroy(S);
      return POISSON_EHIP;
    }
  }
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return POISSON_OK;
}

int poisson_server_submit(poisson_server_t S, int32_t stream_id, int32_t n, const double* d_rho, double* d_phi,
                          void* caller_stream, int64_t* ticket) {
  if (!S || !d_rho || !d_phi || !ticket) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  if (n < 8 || n % 8 != 0 || ((n / 8) & (n / 8 - 1)) != 0) {
    set_error("serving grids need n = 8 * 2^L intervals (got %d)", n);
    return POISSON_EGRID;
  }
  const size_t alone = round_up(plan_bytes(S, n)) + (S->warm ? round_up(phi_bytes(n)) : 0);
  if (alone > S->budget) {
    set_error("request of %zu bytes exceeds the arena of %zu", alone, S->budget);
    return POISSON_EADMIT;
  }
  // order the request after the caller's pending work on rho and phi
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ready, (hipStream_t)caller_stream) != hipSuccess) {
    if (ready) (void)hipEventDestroy(ready);
    set_error("could not record the caller's stream");
    return POISSON_EHIP;
  }
  Request* r = new Request();
  r->stream_id = stream_id;
  r->n = n;
  r->rho = d_rho;
  r->phi = d_phi;
  r->ready = ready;
  r->t_submit = now_ms();
  std::lock_guard<std::mutex> lk(S->mu);
  r->ticket = S->next_ticket++;
  S->reqs[r->ticket] = r;
  S->queue.push_back(r);
  *ticket = r->ticket;
  S->cv.notify_all();
  return POISSON_OK;
}

int poisson_server_poll(poisson_server_t S, int64_t ticket, int32_t* done, poisson_stats_t* stats,
                        double* latency_ms) {
  if (!S || !done) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_error("unknown ticket %lld", (long long)ticket);
    return POISSON_EINVAL;
  }
  Request* r = it->second;
  *done = r->phase == kDone ? 1 : 0;
  if (!*done) return POISSON_OK;
  if (stats) {
    stats->iterations = r->iterations;
    stats->status = r->status;
    stats->rel_residual = r->rel;
    stats->b_norm = r->bnorm;
    stats->rate = (r->iterations > 0 && r->rel > 0.0) ? pow(r->rel, 1.0 / r->iterations) : 0.0;
    stats->t_multipole_ms = 0.0;
    stats->t_iter_ms = r->t_done - r->t_start;
    stats->history_len = 0;
  }
  if (latency_ms) *latency_ms = r->t_done - r->t_submit;
  return r->status;
}

int poisson_server_wait(poisson_server_t S, int64_t ticket, double timeout_ms) {
  if (!S) {
    set_error("null server");
    return POISSON_EINVAL;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_error("unknown ticket %lld", (long long)ticket);
    return POISSON_EINVAL;
  }
  Request* r = it->second;
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double, std::milli>(timeout_ms);
  while (r->phase != kDone)
    if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout && r->phase != kDone) {
      set_error("timed out waiting for ticket %lld", (long long)ticket);
      return POISSON_ETIMEOUT;
    }
  return r->status;
}

int poisson_server_reserve(poisson_server_t S, int32_t n, int32_t count) {
  if (!S || count < 0 || count > kMaxSlots) {
    set_error("bad reservation");
    return POISSON_EINVAL;
  }
  if (n < 8 || n % 8 != 0 || ((n / 8) & (n / 8 - 1)) != 0) {
    set_error("serving grids need n = 8 * 2^L intervals (got %d)", n);
    return POISSON_EGRID;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  S->reserve.emplace_back(n, count);
  ++S->reserve_pending;
  S->reserve_status = POISSON_OK;
  S->cv.notify_all();
  S->cv.wait(lk, [&] { return S->reserve_pending == 0; });
  return S->reserve_status;
}

int poisson_server_footprint(poisson_server_t S, int32_t n, size_t* bytes) {
  if (!S || !bytes) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  *bytes = round_up(plan_bytes(S, n)) + (S->warm ? round_up(phi_bytes(n)) : 0);
  return POISSON_OK;
}

int poisson_server_usage(poisson_server_t S, size_t* used_bytes, int32_t* queued, int32_t* active) {
  if (!S) {
    set_error("null server");
    return POISSON_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (used_bytes) *used_bytes = S->arena.used.load();
  if (queued) *queued = (int32_t)S->queue.size();
  if (active) *active = S->active;
  return POISSON_OK;
}

void poisson_server_destroy(poisson_server_t S) {
  if (!S) return;
  if (S->worker.joinable()) {
    {
      // let queued and running requests finish first
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->queue.empty() && S->active == 0; });
    }
    S->stop.store(true);
    S->cv.notify_all();
    S->worker.join();
  }
  for (int i = 0; i < kMaxSlots; ++i) {
    if (S->streams[i]) (void)hipStreamSynchronize(S->streams[i]);  // the caller's streams stay
    if (S->events[i]) (void)hipEventDestroy(S->events[i]);
  }
  for (PlanEntry* p : S->plans) {
    poisson_plan_destroy(p->plan);
    delete p;
  }
  for (auto& kv : S->reqs)
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
  for (auto& kv : S->reqs) delete kv.second;
  if (S->pinned) (void)hipHostFree(S->pinned);
  delete S;
}

}  // extern "C"
