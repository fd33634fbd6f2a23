// Serving loop for RFD integration requests on one GPU: continuous batching
// under an HBM budget, with resident plans.
//
// Requests wait in a FIFO. A worker thread admits the head whenever an
// in-flight slot is free and the device bytes its plan needs fit the budget
// (evicting idle cached plans, least recently used first), enqueues its work
// on one of a pool of streams and retires it when its event completes. So
// requests that arrive while others run are admitted as slots and memory free
// up, and their kernels overlap on the device.
//
// Plans are cached by their parameters. A request with a nonzero cloud_key
// whose features are resident runs the integrate passes only (B^T F, G = S H,
// expansion); otherwise an idle plan with the same parameters is reused (no
// allocation) or a new one is created, and the one-shot path runs. Work on one
// plan stays on one stream, so requests that share a plan are ordered. The
// phi_1 launches (cooperative grids) of all requests go through one lane
// stream, so two such grids never compete for residency. The request streams
// and the lane together stay within the four hardware queues a process gets
// by default: more streams than queues share queues and serialise behind
// each other's barriers.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rfd_internal.h"

namespace {

constexpr int kMaxInflight = 64;
constexpr int kMaxStreams = 3;  // request streams; with the phi_1 lane, four hardware queues

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool same_params(const rfd_params& a, const rfd_params& b) {
  return a.m == b.m && a.shape == b.shape && a.precision == b.precision && a.eps == b.eps && a.lambda == b.lambda &&
         a.sigma == b.sigma && a.radius == b.radius && a.seed == b.seed && rfd::plan_dim(a) == rfd::plan_dim(b);
}

struct Entry {
  rfd_plan_s* plan = nullptr;
  uint64_t cloud_key = 0;  // cloud whose features the plan holds (0: none to reuse)
  int busy = 0;            // requests in flight on this plan
  int stream = 0;          // stream of its in-flight work
  uint64_t last_use = 0;
};

struct Pending {
  uint64_t ticket;
  rfd_request r;
  double t_submit;
};

struct Slot {
  bool used = false;
  uint64_t ticket = 0;
  Entry* entry = nullptr;
  int stream = 0;
  hipEvent_t done = nullptr, lane_before = nullptr, lane_after = nullptr;
  int* hflag = nullptr;  // pinned host copy of the plan's device flag after the request
  double t_submit = 0, t_start = 0;
};

struct Outcome {
  bool done = false;
  rfd_result res{};
};

}  // namespace

struct rfd_server_s {
  size_t budget = 0;
  int device = 0;
  std::vector<Slot> slots;
  std::vector<hipStream_t> streams;
  std::vector<int> load;  // in-flight requests per stream
  hipStream_t lane = nullptr;
  std::vector<Entry*> entries;
  size_t bytes = 0;  // device bytes of all cached plans
  uint64_t clock = 0;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, Outcome> outcomes;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::thread worker;
};

namespace {

void finish(rfd_server_s* S, uint64_t ticket, rfd_status st, double t_submit, double t_start) {
  Outcome& o = S->outcomes[ticket];
  o.done = true;
  o.res.status = st;
  o.res.t_submit = t_submit;
  o.res.t_start = t_start;
  o.res.t_done = now_s();
  S->cv_done.notify_all();
}

void retire(rfd_server_s* S) {
  for (Slot& sl : S->slots) {
    if (!sl.used) continue;
    const hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) continue;
    rfd_status st = RFD_OK;
    if (e != hipSuccess) {
      st = RFD_ERR_DEVICE;
    } else {
      const int f = *(volatile int*)sl.hflag;
      if (f & 1) st = RFD_ERR_NONFINITE;
      else if (f & 2) st = RFD_ERR_RANGE;
      else if (f & 4) st = RFD_ERR_DEVICE;
    }
    Entry* en = sl.entry;
    --en->busy;
    --S->load[sl.stream];
    if (st != RFD_OK) en->cloud_key = 0;  // do not serve later requests from a failed core
    finish(S, sl.ticket, st, sl.t_submit, sl.t_start);
    sl.used = false;
    sl.entry = nullptr;
  }
}

void evict(rfd_server_s* S, Entry* e) {
  S->bytes -= rfd::plan_device_bytes(e->plan);
  rfd::free_plan_device(e->plan);
  for (size_t i = 0; i < S->entries.size(); ++i)
    if (S->entries[i] == e) {
      S->entries.erase(S->entries.begin() + (long)i);
      break;
    }
  delete e;
}

size_t grow_bytes(const rfd_plan_s* p, int64_t N, size_t partial_floats, bool copies_x) {
  size_t g = 0;
  if (copies_x && N > p->dev.Xcap) g += sizeof(float) * 3 * (size_t)(N - p->dev.Xcap);
  if (partial_floats > p->dev.partials_cap) g += sizeof(float) * (partial_floats - p->dev.partials_cap);
  return g;
}

// Tries to start the request at the head of the queue. Returns false when it
// has to wait (no free slot, or its bytes do not fit even after evicting every
// idle plan); true when it was started or finished with an error.
bool admit_head(rfd_server_s* S) {
  int si = -1;
  for (int i = 0; i < (int)S->slots.size(); ++i)
    if (!S->slots[i].used) {
      si = i;
      break;
    }
  if (si < 0) return false;
  const Pending q = S->queue.front();
  const rfd_request& r = q.r;
  const int M = rfd::padded_m(r.params.m), prec = r.params.precision;
  Entry* e = nullptr;
  bool resident = false;
  if (r.cloud_key)
    for (Entry* c : S->entries)
      if (c->cloud_key == r.cloud_key && c->plan->N == r.N && same_params(c->plan->params, r.params)) {
        e = c;
        resident = true;
        break;
      }
  const size_t pf = rfd::request_partial_floats(M, prec, r.N, r.d, !resident);
  const size_t need_new = rfd::plan_fixed_bytes(M) + sizeof(float) * 3 * (size_t)r.N + sizeof(float) * pf;
  // a new cloud takes an idle plan with the same parameters that holds no
  // features worth keeping; else a new plan while the budget allows; else
  // the least recently used idle plan with the same parameters
  for (int pass = 0; !e && pass < 2; ++pass) {
    if (pass == 1 && S->bytes + need_new <= S->budget) break;
    for (Entry* c : S->entries)
      if (c->busy == 0 && same_params(c->plan->params, r.params) && (pass == 1 || c->cloud_key == 0) &&
          (!e || c->last_use < e->last_use))
        e = c;
  }
  size_t need = e ? grow_bytes(e->plan, r.N, pf, !resident) : need_new;
  if (e && need > 0 && e->busy) return false;  // a busy plan grows only once idle
  while (S->bytes + need > S->budget) {
    Entry* victim = nullptr;
    for (Entry* c : S->entries)
      if (c != e && c->busy == 0 && (!victim || c->last_use < victim->last_use)) victim = c;
    if (!victim) return false;
    evict(S, victim);
  }
  S->queue.pop_front();
  const double t_start = now_s();
  if (!e) {
    rfd_plan_t p = nullptr;
    const rfd_status cs = rfd_plan_create(&r.params, &p);
    if (cs != RFD_OK) {
      finish(S, q.ticket, cs, q.t_submit, t_start);
      return true;
    }
    e = new Entry();
    e->plan = p;
    S->entries.push_back(e);
    S->bytes += rfd::plan_device_bytes(p);
  }
  int sidx = e->stream;
  if (e->busy == 0) {
    sidx = 0;
    for (int i = 1; i < (int)S->streams.size(); ++i)
      if (S->load[i] < S->load[sidx]) sidx = i;
  }
  hipStream_t st = S->streams[sidx];
  Slot& sl = S->slots[si];
  const size_t before = rfd::plan_device_bytes(e->plan);
  rfd_status s;
  if (resident) {
    s = rfd::integrate_enqueue(e->plan, r.F, r.ldF, r.d, r.out, r.ldO, st, 0, nullptr);
  } else {
    const rfd::PhiLane lane{S->lane, sl.lane_before, sl.lane_after};
    s = rfd::oneshot_enqueue(e->plan, r.X, r.N, r.F, r.ldF, r.d, r.out, r.ldO, st, &lane);
    e->cloud_key = s == RFD_OK ? r.cloud_key : 0;
  }
  S->bytes += rfd::plan_device_bytes(e->plan) - before;
  if (s == RFD_OK &&
      (hipMemcpyAsync(sl.hflag, e->plan->dev.flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipMemsetAsync(e->plan->dev.flag, 0, sizeof(int), st) != hipSuccess || hipEventRecord(sl.done, st) != hipSuccess))
    s = RFD_ERR_DEVICE;
  if (s != RFD_OK) {
    // part of the work may have been enqueued: let it drain before the plan is reused
    (void)hipStreamSynchronize(st);
    e->cloud_key = 0;
    finish(S, q.ticket, s, q.t_submit, t_start);
    return true;
  }
  sl.used = true;
  sl.ticket = q.ticket;
  sl.entry = e;
  sl.stream = sidx;
  sl.t_submit = q.t_submit;
  sl.t_start = t_start;
  ++e->busy;
  e->stream = sidx;
  e->last_use = ++S->clock;
  ++S->load[sidx];
  return true;
}

void worker_main(rfd_server_s* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    retire(S);
    if (S->stop) {
      while (!S->queue.empty()) {
        finish(S, S->queue.front().ticket, RFD_ERR_SHUTDOWN, S->queue.front().t_submit, 0.0);
        S->queue.pop_front();
      }
    } else {
      while (!S->queue.empty() && admit_head(S)) {
      }
    }
    bool inflight = false;
    for (const Slot& sl : S->slots) inflight = inflight || sl.used;
    if (S->stop && !inflight) break;
    if (inflight) {
      S->cv_work.wait_for(lk, std::chrono::microseconds(20));
    } else if (S->queue.empty()) {
      S->cv_work.wait(lk);
    } else {
      S->cv_work.wait_for(lk, std::chrono::milliseconds(1));
    }
  }
}

void destroy_server(rfd_server_s* S) {
  (void)hipDeviceSynchronize();
  for (Entry* e : S->entries) {
    rfd::free_plan_device(e->plan);
    delete e;
  }
  S->entries.clear();
  for (Slot& sl : S->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.lane_before) (void)hipEventDestroy(sl.lane_before);
    if (sl.lane_after) (void)hipEventDestroy(sl.lane_after);
    if (sl.hflag) (void)hipHostFree(sl.hflag);
  }
  for (hipStream_t s : S->streams)
    if (s) (void)hipStreamDestroy(s);
  if (S->lane) (void)hipStreamDestroy(S->lane);
  delete S;
}

}  // namespace

extern "C" {

rfd_status rfd_server_create(size_t hbm_budget_bytes, int32_t max_inflight, rfd_server_t* out) {
  if (!out) return RFD_ERR_INVALID_ARG;
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_inflight < 1 || max_inflight > kMaxInflight) return RFD_ERR_INVALID_ARG;
  rfd_server_s* S = new (std::nothrow) rfd_server_s();
  if (!S) return RFD_ERR_DEVICE;
  S->budget = hbm_budget_bytes;
  bool ok = hipGetDevice(&S->device) == hipSuccess;
  const int ns = max_inflight < kMaxStreams ? max_inflight : kMaxStreams;
  S->streams.assign(ns, nullptr);
  S->load.assign(ns, 0);
  for (int i = 0; ok && i < ns; ++i) ok = hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&S->lane, hipStreamNonBlocking) == hipSuccess;
  S->slots.resize(max_inflight);
  for (Slot& sl : S->slots) {
    ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.lane_before, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.lane_after, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc((void**)&sl.hflag, sizeof(int), hipHostMallocDefault) == hipSuccess;
    if (ok) *sl.hflag = 0;
  }
  if (!ok) {
    destroy_server(S);
    return RFD_ERR_DEVICE;
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return RFD_OK;
}

rfd_status rfd_submit(rfd_server_t S, const rfd_request* r, uint64_t* ticket) {
  if (!S || !r || !ticket) return RFD_ERR_INVALID_ARG;
  *ticket = 0;
  rfd_status s = rfd::check_params(&r->params);
  if (s != RFD_OK) return s;
  if (r->params.omega || rfd::plan_dim(r->params) != 3 || r->N < 0 || (r->N > 0 && !r->X)) return RFD_ERR_INVALID_ARG;
  s = rfd::check_field_args(r->N, r->F, r->ldF, r->d, r->out, r->ldO);
  if (s != RFD_OK) return s;
  const int M = rfd::padded_m(r->params.m);
  const size_t need = rfd::plan_fixed_bytes(M) + sizeof(float) * 3 * (size_t)r->N +
                      sizeof(float) * rfd::request_partial_floats(M, r->params.precision, r->N, r->d, true);
  if (need > S->budget) return RFD_ERR_OUT_OF_BUDGET;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return RFD_ERR_SHUTDOWN;
  const uint64_t t = S->next_ticket++;
  const double now = now_s();
  S->outcomes[t] = Outcome{};
  if (r->N == 0 || r->d == 0) {
    finish(S, t, RFD_OK, now, now);  // nothing to integrate
  } else {
    S->queue.push_back(Pending{t, *r, now});
    S->cv_work.notify_one();
  }
  *ticket = t;
  return RFD_OK;
}

rfd_status rfd_wait(rfd_server_t S, uint64_t ticket, double timeout_s, rfd_result* res) {
  if (!S) return RFD_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->outcomes.find(ticket);
  if (it == S->outcomes.end()) return RFD_ERR_INVALID_ARG;
  Outcome& o = it->second;  // element references survive rehashing
  if (timeout_s < 0) {
    S->cv_done.wait(lk, [&] { return o.done; });
  } else {
    S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return o.done; });
  }
  if (!o.done) return RFD_ERR_NOT_READY;
  const rfd_result out = o.res;
  S->outcomes.erase(ticket);
  if (res) *res = out;
  return out.status;
}

rfd_status rfd_server_stats(rfd_server_t S, size_t* device_bytes, int32_t* plans, int32_t* queued,
                            int32_t* inflight) {
  if (!S) return RFD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(S->mu);
  int nin = 0;
  for (const Slot& sl : S->slots) nin += sl.used ? 1 : 0;
  if (device_bytes) *device_bytes = S->bytes;
  if (plans) *plans = (int32_t)S->entries.size();
  if (queued) *queued = (int32_t)S->queue.size();
  if (inflight) *inflight = nin;
  return RFD_OK;
}

void rfd_server_destroy(rfd_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  destroy_server(S);
}

}  // extern "C"
