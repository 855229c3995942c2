// Continuous-batching server for negacyclic polynomial products.
//
// A request is c = a * b in Z_q[X]/(X^N + 1) for each of its RNS limbs: the
// forward transform of both factors, the dyadic modular product and the
// inverse transform of the Section 4 product listing, per limb (limbs are
// independent, Section 5).  The scheduler thread owns every queue:
//   future   -- submitted, arrival time not reached (min-heap on arrival);
//   ready    -- arrived, waiting for arena space (arrival order);
//   admitted -- arena space reserved, not launched;
// launches in flight sit in stream slots (persistent batch launches), in a
// list of per-request events on the wide streams (batched mode, large rings:
// a limb product of N >= 2^15 inside one workgroup would take milliseconds,
// while the two-pass kernels spread it over the chip), or in an in-order list
// of per-request events (FIFO modes).  Host time stamps use the
// monotonic clock; a request's completion time is taken when the scheduler
// sees the event of the launch holding it complete (it polls while work is
// in flight).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <queue>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace nttamd {
namespace {

int64_t clock_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr uint64_t kArenaAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kArenaAlign - 1) & ~(kArenaAlign - 1); }

// First-fit allocator over the byte range [0, size) of the device arena;
// adjacent free ranges are merged on release.  Host bookkeeping only.
class Arena {
 public:
  void init(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = peak_ = 0;
  }
  bool alloc(uint64_t len, uint64_t* off) {
    len = align_up(len);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      const uint64_t rest = it->second - len, start = it->first + len;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += len;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t len) {
    len = align_up(len);
    used_ -= len;
    uint64_t start = off, end = off + len;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && next->first == end) {
      end += next->second;
      free_.erase(next);
    }
    free_[start] = end - start;
  }
  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }

 private:
  std::map<uint64_t, uint64_t> free_;   // offset -> length
  uint64_t size_ = 0, used_ = 0, peak_ = 0;
};

struct Req {
  uint64_t ticket = 0;
  uint64_t N = 0;
  uint32_t L = 0, logN = 0;
  const uint64_t* a = nullptr;
  const uint64_t* b = nullptr;
  std::vector<const ntt_plan*> plans;
  std::vector<uint64_t> moduli;
  int64_t arrival = 0, admit = 0, launch = 0, done = 0;
  uint64_t out_off = 0, out_len = 0, tmp_off = 0, tmp_len = 0;
  bool has_out = false, has_tmp = false, deferred = false;
  uint32_t state = NTT_REQ_WAITING;
  ntt_status status = NTT_OK;
  std::vector<hipEvent_t> read_events;   // one per ntt_server_read: the copy's completion on the caller's stream
};

// Arena ranges whose last users are still on the device: freed once every
// event has completed (reads on callers' streams, or a failed request's
// already-enqueued kernels).
struct PendingFree {
  std::vector<hipEvent_t> events;
  uint64_t off[2] = {0, 0}, len[2] = {0, 0};
};

struct LaterArrival {
  bool operator()(const Req* x, const Req* y) const {
    return x->arrival != y->arrival ? x->arrival > y->arrival : x->ticket > y->ticket;
  }
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  ntt_batch* batch = nullptr;
  std::vector<Req*> reqs;
  bool busy = false;
};

}  // namespace
}  // namespace nttamd

using namespace nttamd;

struct ntt_server {
  int device = 0;
  ntt_server_config cfg{};
  uint64_t* base = nullptr;      // device arena
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler: new submission, release, stop
  std::condition_variable cv_done;   // waiters: completions
  std::thread thread;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t outstanding = 0;          // submitted and neither done nor failed
  std::unordered_map<uint64_t, std::unique_ptr<Req>> records;
  std::priority_queue<Req*, std::vector<Req*>, LaterArrival> future;
  std::deque<Req*> ready;
  std::deque<Req*> admitted;        // to the persistent batch launches
  std::deque<Req*> admitted_wide;   // batched mode, N >= 2^wide_min: own launches on the wide streams
  std::vector<hipStream_t> wide;
  size_t wide_rr = 0;
  std::vector<std::pair<hipEvent_t, Req*>> wide_inflight;
  std::vector<Slot> slots;
  std::deque<std::pair<hipEvent_t, Req*>> fifo_inflight;
  std::vector<hipEvent_t> event_pool;
  std::vector<PendingFree> pending_free;
  std::vector<BatchTask> tasks;
  ntt_server_stats st{};
};

namespace nttamd {
namespace {

uint64_t result_bytes(const ntt_server* s, uint64_t N, uint32_t L) {
  (void)s;
  return align_up((uint64_t)L * N * sizeof(uint64_t));
}
uint64_t workspace_bytes(const ntt_server* s, uint64_t N, uint32_t L, uint32_t logN) {
  if (s->cfg.mode == NTT_SERVE_FIFO_PER_LIMB) return align_up(N * sizeof(uint64_t));
  return logN > (uint32_t)kMaxOnchipLog ? align_up((uint64_t)L * N * sizeof(uint64_t)) : 0;
}

bool reserve(ntt_server* s, Req* r) {
  if (!s->arena.alloc(r->out_len, &r->out_off)) return false;
  if (r->tmp_len && !s->arena.alloc(r->tmp_len, &r->tmp_off)) {
    s->arena.release(r->out_off, r->out_len);
    return false;
  }
  r->has_out = true;
  r->has_tmp = r->tmp_len != 0;
  return true;
}

void drop_tmp(ntt_server* s, Req* r) {
  if (r->has_tmp) s->arena.release(r->tmp_off, r->tmp_len);
  r->has_tmp = false;
}
void drop_out(ntt_server* s, Req* r) {
  if (r->has_out) s->arena.release(r->out_off, r->out_len);
  r->has_out = false;
}

hipEvent_t take_event(ntt_server* s);

// Frees the request's arena ranges once `stream` has drained the work already
// enqueued on it (an event, or a synchronisation when no event can be had).
void free_after(ntt_server* s, Req* r, hipStream_t stream) {
  PendingFree pf;
  int k = 0;
  if (r->has_out) { pf.off[k] = r->out_off; pf.len[k++] = r->out_len; }
  if (r->has_tmp) { pf.off[k] = r->tmp_off; pf.len[k++] = r->tmp_len; }
  r->has_out = r->has_tmp = false;
  if (!k) return;
  hipEvent_t ev = take_event(s);
  if (ev && hipEventRecord(ev, stream) == hipSuccess) {
    pf.events.push_back(ev);
    s->pending_free.push_back(std::move(pf));
    return;
  }
  if (ev) s->event_pool.push_back(ev);
  (void)hipStreamSynchronize(stream);
  for (int i = 0; i < k; ++i) s->arena.release(pf.off[i], pf.len[i]);
}

// stream: where the request's kernels were enqueued when a launch failed part
// way (nullptr when nothing of it reached the device, or on completion).
void finish(ntt_server* s, Req* r, int64_t t, ntt_status status, hipStream_t stream = nullptr) {
  r->done = t;
  r->status = status;
  r->state = status == NTT_OK ? NTT_REQ_DONE : NTT_REQ_FAILED;
  if (status != NTT_OK && stream) {
    free_after(s, r, stream);        // earlier launches of this request may still write its ranges
  } else {
    drop_tmp(s, r);
    if (status != NTT_OK || s->cfg.release_on_completion) drop_out(s, r);
  }
  if (status == NTT_OK) ++s->st.completed;
  else ++s->st.failed;
  --s->outstanding;
}

// Returns the ranges whose events have all completed to the arena.
bool reap_frees(ntt_server* s) {
  bool any = false;
  for (size_t i = 0; i < s->pending_free.size();) {
    PendingFree& pf = s->pending_free[i];
    bool done = true;
    for (hipEvent_t e : pf.events)
      if (hipEventQuery(e) == hipErrorNotReady) { done = false; break; }
    if (!done) { ++i; continue; }
    for (int k = 0; k < 2; ++k)
      if (pf.len[k]) s->arena.release(pf.off[k], pf.len[k]);
    for (hipEvent_t e : pf.events) s->event_pool.push_back(e);
    pf = std::move(s->pending_free.back());
    s->pending_free.pop_back();
    any = true;
  }
  return any;
}

void admit(ntt_server* s) {
  while (!s->ready.empty()) {
    Req* r = s->ready.front();
    if (!reserve(s, r)) {
      if (!r->deferred) {
        r->deferred = true;
        ++s->st.deferred;
      }
      return;                                      // strict arrival order: the head blocks the rest
    }
    r->state = NTT_REQ_ADMITTED;
    r->admit = clock_ns();
    if (s->cfg.mode == NTT_SERVE_BATCHED && r->logN >= s->cfg.wide_min_log_degree) s->admitted_wide.push_back(r);
    else s->admitted.push_back(r);
    s->ready.pop_front();
  }
}

hipEvent_t take_event(ntt_server* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Forward / multiply / inverse of one request as three launches over its limbs.
ntt_status enqueue_fused(ntt_server* s, Req* r, hipStream_t stream) {
  uint64_t* out = s->base + r->out_off / sizeof(uint64_t);
  uint64_t* tmp = r->has_tmp ? s->base + r->tmp_off / sizeof(uint64_t) : nullptr;
  NttLaunch l{};
  l.plans = r->plans.data();
  l.num_limbs = r->L;
  l.num_polys = 1;
  l.stream = stream;
  l.out = out;
  l.in = r->a;
  l.in_f = 1;
  l.out_f = 4;
  ntt_status e = launch_forward(l);                 // out <- NTT(a), [0, 4q)
  if (e) return e;
  l.in = r->b;
  l.mul_into = out;
  l.tmp = tmp;
  e = launch_forward(l);                            // out <- NTT(b) (.) out, canonical
  if (e) return e;
  l.in = out;
  l.mul_into = nullptr;
  l.tmp = nullptr;
  l.out_f = 1;
  return launch_inverse(l);                         // out <- InvNTT(out), canonical
}

// The plain form: per limb, forward(a), forward(b), multiply, inverse.
ntt_status enqueue_per_limb(ntt_server* s, Req* r, hipStream_t stream) {
  uint64_t* out = s->base + r->out_off / sizeof(uint64_t);
  uint64_t* tmp = s->base + r->tmp_off / sizeof(uint64_t);
  for (uint32_t l = 0; l < r->L; ++l) {
    uint64_t* ol = out + (uint64_t)l * r->N;
    NttLaunch f{};
    f.plans = &r->plans[l];
    f.num_limbs = 1;
    f.num_polys = 1;
    f.stream = stream;
    f.in_f = 1;
    f.out_f = 4;
    f.out = ol;
    f.in = r->a + (uint64_t)l * r->N;
    ntt_status e = launch_forward(f);
    if (e) return e;
    f.out = tmp;
    f.in = r->b + (uint64_t)l * r->N;
    e = launch_forward(f);
    if (e) return e;
    EltLaunch m{};
    m.out = ol;
    m.a = ol;
    m.b = tmp;
    m.n = r->N;
    m.moduli = &r->moduli[l];
    m.num_limbs = 1;
    m.num_polys = 1;
    m.in_f = 4;
    m.stream = stream;
    e = launch_eltwise_mult(m);
    if (e) return e;
    f.out = ol;
    f.in = ol;
    f.out_f = 1;
    e = launch_inverse(f);
    if (e) return e;
  }
  return NTT_OK;
}

bool launch(ntt_server* s) {
  bool any = false;
  if (s->cfg.mode == NTT_SERVE_BATCHED) {
    // large rings: the wide two-pass kernels, three launches over the request's limbs,
    // round robin over the wide streams (they overlap the persistent launches)
    // While the wide streams already hold wide_max_inflight launches each, further large
    // requests join the persistent launches instead: under load the packed
    // launch keeps the chip fuller than more separate launches would.
    const size_t wide_cap = (size_t)s->cfg.wide_max_inflight * s->wide.size();
    while (!s->admitted_wide.empty() && s->wide_inflight.size() >= wide_cap) {
      s->admitted.push_back(s->admitted_wide.front());
      s->admitted_wide.pop_front();
    }
    while (!s->admitted_wide.empty()) {
      Req* r = s->admitted_wide.front();
      s->admitted_wide.pop_front();
      hipStream_t ws = s->wide[s->wide_rr++ % s->wide.size()];
      r->state = NTT_REQ_RUNNING;
      r->launch = clock_ns();
      ntt_status e = enqueue_fused(s, r, ws);
      hipEvent_t ev = e ? nullptr : take_event(s);
      if (!e && (!ev || hipEventRecord(ev, ws) != hipSuccess)) e = NTT_EDEVICE;
      if (e) {
        if (ev) s->event_pool.push_back(ev);
        finish(s, r, clock_ns(), e, ws);
        s->cv_done.notify_all();
        continue;
      }
      s->wide_inflight.emplace_back(ev, r);
      ++s->st.launches;
      s->st.tasks += r->L;
      any = true;
      while (!s->admitted_wide.empty() && s->wide_inflight.size() >= wide_cap) {
        s->admitted.push_back(s->admitted_wide.front());
        s->admitted_wide.pop_front();
      }
    }
    const size_t cap = s->cfg.max_batch_tasks;
    for (Slot& sl : s->slots) {
      if (s->admitted.empty()) break;
      if (sl.busy) continue;
      s->tasks.clear();
      sl.reqs.clear();
      while (!s->admitted.empty()) {
        Req* r = s->admitted.front();
        if (s->tasks.size() + r->L > cap) break;
        uint64_t* out = s->base + r->out_off / sizeof(uint64_t);
        uint64_t* tmp = r->has_tmp ? s->base + r->tmp_off / sizeof(uint64_t) : nullptr;
        for (uint32_t l = 0; l < r->L; ++l) {
          BatchTask t{};
          const uint64_t off = (uint64_t)l * r->N;
          t.out = out + off;
          t.in = r->a + off;
          t.in2 = r->b + off;
          t.tmp = tmp ? tmp + off : nullptr;
          t.plan = r->plans[l]->dev;
          t.logN = r->logN;
          t.op = kBatchProduct | batch_wide_flag(r->logN, r->moduli[l]);
          s->tasks.push_back(t);
        }
        r->state = NTT_REQ_RUNNING;
        sl.reqs.push_back(r);
        s->admitted.pop_front();
      }
      const int64_t t = clock_ns();
      for (Req* r : sl.reqs) r->launch = t;
      ntt_status e = batch_launch_tasks(sl.batch, s->tasks.data(), s->tasks.size(), sl.stream, s->cfg.use_graph != 0);
      if (e == NTT_OK && hipEventRecord(sl.event, sl.stream) != hipSuccess) e = NTT_EDEVICE;
      if (e) {
        for (Req* r : sl.reqs) finish(s, r, clock_ns(), e, sl.stream);
        sl.reqs.clear();
        s->cv_done.notify_all();
        continue;
      }
      sl.busy = true;
      ++s->st.launches;
      s->st.tasks += s->tasks.size();
      any = true;
    }
    return any;
  }
  hipStream_t stream = s->slots[0].stream;
  while (!s->admitted.empty()) {
    Req* r = s->admitted.front();
    s->admitted.pop_front();
    r->state = NTT_REQ_RUNNING;
    r->launch = clock_ns();
    ntt_status e = s->cfg.mode == NTT_SERVE_FIFO ? enqueue_fused(s, r, stream) : enqueue_per_limb(s, r, stream);
    hipEvent_t ev = e ? nullptr : take_event(s);
    if (!e && (!ev || hipEventRecord(ev, stream) != hipSuccess)) e = NTT_EDEVICE;
    if (e) {
      if (ev) s->event_pool.push_back(ev);
      finish(s, r, clock_ns(), e, stream);
      s->cv_done.notify_all();
      continue;
    }
    s->fifo_inflight.emplace_back(ev, r);
    ++s->st.launches;
    s->st.tasks += r->L;
    any = true;
  }
  return any;
}

bool reap(ntt_server* s) {
  bool any = false;
  for (Slot& sl : s->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.event);
    if (q == hipErrorNotReady) continue;
    const int64_t t = clock_ns();
    for (Req* r : sl.reqs) finish(s, r, t, q == hipSuccess ? NTT_OK : NTT_EDEVICE);
    sl.reqs.clear();
    sl.busy = false;
    any = true;
  }
  for (size_t i = 0; i < s->wide_inflight.size();) {
    auto& f = s->wide_inflight[i];
    const hipError_t q = hipEventQuery(f.first);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    finish(s, f.second, clock_ns(), q == hipSuccess ? NTT_OK : NTT_EDEVICE);
    s->event_pool.push_back(f.first);
    f = s->wide_inflight.back();
    s->wide_inflight.pop_back();
    any = true;
  }
  while (!s->fifo_inflight.empty()) {
    auto& f = s->fifo_inflight.front();
    const hipError_t q = hipEventQuery(f.first);
    if (q == hipErrorNotReady) break;
    finish(s, f.second, clock_ns(), q == hipSuccess ? NTT_OK : NTT_EDEVICE);
    s->event_pool.push_back(f.first);
    s->fifo_inflight.pop_front();
    any = true;
  }
  if (any) s->cv_done.notify_all();
  return reap_frees(s) || any;
}

bool in_flight(const ntt_server* s) {
  if (!s->fifo_inflight.empty() || !s->wide_inflight.empty() || !s->pending_free.empty()) return true;
  for (const Slot& sl : s->slots)
    if (sl.busy) return true;
  return false;
}

void cancel_pending(ntt_server* s) {
  const int64_t t = clock_ns();
  while (!s->future.empty()) {
    finish(s, s->future.top(), t, NTT_EBUSY);
    s->future.pop();
  }
  for (Req* r : s->ready) finish(s, r, t, NTT_EBUSY);
  s->ready.clear();
  for (Req* r : s->admitted) finish(s, r, t, NTT_EBUSY);
  s->admitted.clear();
  for (Req* r : s->admitted_wide) finish(s, r, t, NTT_EBUSY);
  s->admitted_wide.clear();
  s->cv_done.notify_all();
}

void scheduler(ntt_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    const int64_t now = clock_ns();
    while (!s->future.empty() && s->future.top()->arrival <= now) {
      s->ready.push_back(s->future.top());
      s->future.pop();
    }
    if (s->stop) cancel_pending(s);
    admit(s);
    bool progressed = launch(s);
    progressed = reap(s) || progressed;
    const bool busy = in_flight(s);
    if (s->stop && !busy) break;
    if (progressed) continue;
    if (busy) {                                    // poll the device while work is in flight
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
      continue;
    }
    if (!s->ready.empty() || s->future.empty()) {  // waiting for a release, a submission or stop
      s->cv_work.wait(lk);
      continue;
    }
    const int64_t wait = s->future.top()->arrival - clock_ns();
    constexpr int64_t kSpinNs = 200000;            // sleep until shortly before the next arrival, then spin
    if (wait > kSpinNs) {
      s->cv_work.wait_for(lk, std::chrono::nanoseconds(wait - kSpinNs));
    } else {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
}

void fill_info(const ntt_server* s, const Req* r, ntt_request_info* info) {
  info->state = r->state;
  info->status = r->status;
  info->result = (r->state == NTT_REQ_DONE && r->has_out) ? s->base + r->out_off / sizeof(uint64_t) : nullptr;
  info->arrival_ns = r->arrival;
  info->admit_ns = r->admit;
  info->launch_ns = r->launch;
  info->done_ns = r->done;
}

void destroy_resources(ntt_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.batch) (void)ntt_batch_destroy(sl.batch);
    if (sl.event) (void)hipEventDestroy(sl.event);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (hipStream_t w : s->wide) (void)hipStreamDestroy(w);
  for (PendingFree& pf : s->pending_free)
    for (hipEvent_t e : pf.events) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  s->pending_free.clear();
  for (auto& kv : s->records)
    for (hipEvent_t e : kv.second->read_events) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  if (s->base) (void)hipFree(s->base);
}

}  // namespace
}  // namespace nttamd

extern "C" {

int64_t ntt_server_now_ns(void) { return clock_ns(); }

ntt_status ntt_server_create(ntt_server** out, const ntt_server_config* config) {
  if (!out) return NTT_EINVAL_POINTER;
  *out = nullptr;
  ntt_server_config c{};
  if (config) c = *config;
  if (c.mode > NTT_SERVE_FIFO_PER_LIMB) return NTT_EINVAL_COUNT;
  if (c.hbm_budget == 0) c.hbm_budget = 16ull << 30;
  if (c.streams == 0) c.streams = 2;
  if (c.streams > 4) return NTT_EINVAL_COUNT;
  if (c.max_batch_tasks == 0) c.max_batch_tasks = 4096;
  if (c.max_batch_tasks < NTT_MAX_LIMBS || c.max_batch_tasks > (1u << 20)) return NTT_EINVAL_COUNT;
  if (c.max_queue == 0) c.max_queue = 1u << 20;
  if (c.wide_min_log_degree == 0) c.wide_min_log_degree = kMaxOnchipLog + 1;
  if (c.wide_max_inflight == 0) c.wide_max_inflight = 2;
  if (c.wide_max_inflight > 1024) return NTT_EINVAL_COUNT;
  if (c.wide_min_log_degree < 10 || c.wide_min_log_degree > NTT_MAX_LOG_DEGREE + 1) return NTT_EINVAL_COUNT;
  c.hbm_budget = align_up(c.hbm_budget);
  std::unique_ptr<ntt_server> s(new (std::nothrow) ntt_server());
  if (!s) return NTT_ENOMEM;
  s->cfg = c;
  if (hipGetDevice(&s->device) != hipSuccess) return NTT_EDEVICE;
  if (hipMalloc((void**)&s->base, c.hbm_budget) != hipSuccess) {
    s->base = nullptr;
    return NTT_ENOMEM;
  }
  s->arena.init(c.hbm_budget);
  const uint32_t nslots = c.mode == NTT_SERVE_BATCHED ? c.streams : 1;
  s->slots.resize(nslots);
  for (Slot& sl : s->slots) {
    ntt_status e = NTT_OK;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.event, hipEventDisableTiming) != hipSuccess)
      e = NTT_EDEVICE;
    if (!e && c.mode == NTT_SERVE_BATCHED) e = ntt_batch_create(&sl.batch, c.max_batch_tasks);
    // the server's slots already spread over the hardware queues: no extra copy stream per slot
    if (!e && sl.batch) batch_use_copy_stream(sl.batch, false);
    if (e) {
      destroy_resources(s.get());
      return e;
    }
  }
  if (c.mode == NTT_SERVE_BATCHED) {
    s->wide.resize(c.streams, nullptr);
    for (hipStream_t& w : s->wide) {
      if (hipStreamCreateWithFlags(&w, hipStreamNonBlocking) != hipSuccess) {
        w = nullptr;
        destroy_resources(s.get());
        return NTT_EDEVICE;
      }
    }
  }
  try {
    s->thread = std::thread(scheduler, s.get());
  } catch (...) {
    destroy_resources(s.get());
    return NTT_ENOMEM;
  }
  *out = s.release();
  return NTT_OK;
}

ntt_status ntt_server_submit(ntt_server* s, const ntt_request* q, uint64_t* ticket) {
  if (!s) return NTT_EINVAL_POINTER;
  auto reject = [s](ntt_status e) {
    std::lock_guard<std::mutex> g(s->mu);
    ++s->st.rejected;
    return e;
  };
  if (ticket) *ticket = 0;
  if (!q || !ticket || !q->a || !q->b || !q->moduli) return reject(NTT_EINVAL_POINTER);
  ntt_status e = validate_degree(q->N);
  if (e) return reject(e);
  if (q->N < 1024) return reject(NTT_EINVAL_DEGREE);
  if (q->num_limbs == 0 || q->num_limbs > NTT_MAX_LIMBS) return reject(NTT_EINVAL_COUNT);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->device) return reject(NTT_EDEVICE);
  std::unique_ptr<Req> r(new (std::nothrow) Req());
  if (!r) return reject(NTT_ENOMEM);
  r->N = q->N;
  r->L = (uint32_t)q->num_limbs;
  while ((1ull << r->logN) < r->N) ++r->logN;
  r->a = q->a;
  r->b = q->b;
  r->out_len = result_bytes(s, r->N, r->L);
  r->tmp_len = workspace_bytes(s, r->N, r->L, r->logN);
  if (r->out_len + r->tmp_len > s->arena.size()) return reject(NTT_ENOMEM);
  r->moduli.assign(q->moduli, q->moduli + r->L);
  r->plans.resize(r->L);
  for (uint32_t l = 0; l < r->L; ++l) {
    const ntt_plan* p = nullptr;
    e = cached_plan(r->N, r->moduli[l], &p);
    if (e) return reject(e);
    r->plans[l] = p;
  }
  if (validate_enabled()) {
    e = check_range(q->a, 64, q->N, q->moduli, q->num_limbs, 1, 1, nullptr);
    if (!e) e = check_range(q->b, 64, q->N, q->moduli, q->num_limbs, 1, 1, nullptr);
    if (e) return reject(e);
  }
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) {
    ++s->st.rejected;
    return NTT_EBUSY;
  }
  if (s->future.size() + s->ready.size() >= s->cfg.max_queue) {
    ++s->st.rejected;
    return NTT_EBUSY;
  }
  r->ticket = s->next_ticket++;
  r->arrival = q->arrival_ns ? q->arrival_ns : clock_ns();
  Req* raw = r.get();
  s->records.emplace(raw->ticket, std::move(r));
  s->future.push(raw);
  ++s->outstanding;
  ++s->st.submitted;
  *ticket = raw->ticket;
  s->cv_work.notify_one();
  return NTT_OK;
}

ntt_status ntt_server_poll(ntt_server* s, uint64_t ticket, ntt_request_info* info) {
  if (!s || !info) return NTT_EINVAL_POINTER;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->records.find(ticket);
  if (it == s->records.end()) return NTT_ENOTFOUND;
  fill_info(s, it->second.get(), info);
  return NTT_OK;
}

ntt_status ntt_server_query(ntt_server* s, const uint64_t* tickets, size_t count, ntt_request_info* infos) {
  if (!s || ((!tickets || !infos) && count)) return NTT_EINVAL_POINTER;
  std::lock_guard<std::mutex> g(s->mu);
  for (size_t i = 0; i < count; ++i) {
    auto it = s->records.find(tickets[i]);
    if (it == s->records.end()) return NTT_ENOTFOUND;
    fill_info(s, it->second.get(), &infos[i]);
  }
  return NTT_OK;
}

ntt_status ntt_server_wait(ntt_server* s, uint64_t ticket, int64_t timeout_ns, ntt_request_info* info) {
  if (!s) return NTT_EINVAL_POINTER;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->records.find(ticket);
  if (it == s->records.end()) return NTT_ENOTFOUND;
  Req* r = it->second.get();
  auto finished = [r] { return r->state == NTT_REQ_DONE || r->state == NTT_REQ_FAILED; };
  if (timeout_ns < 0) s->cv_done.wait(lk, finished);
  else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), finished)) return NTT_ETIMEDOUT;
  if (info) fill_info(s, r, info);
  return NTT_OK;
}

ntt_status ntt_server_drain(ntt_server* s, int64_t timeout_ns) {
  if (!s) return NTT_EINVAL_POINTER;
  std::unique_lock<std::mutex> lk(s->mu);
  auto idle = [s] { return s->outstanding == 0; };
  if (timeout_ns < 0) s->cv_done.wait(lk, idle);
  else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), idle)) return NTT_ETIMEDOUT;
  return NTT_OK;
}

ntt_status ntt_server_read(ntt_server* s, uint64_t ticket, uint64_t* dst, ntt_stream_t stream) {
  if (!s || !dst) return NTT_EINVAL_POINTER;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->records.find(ticket);
  if (it == s->records.end()) return NTT_ENOTFOUND;
  Req* r = it->second.get();
  if (r->state == NTT_REQ_FAILED) return r->status;
  if (r->state != NTT_REQ_DONE) return NTT_EBUSY;
  if (!r->has_out) return NTT_ENOTFOUND;
  const size_t bytes = (size_t)r->L * r->N * sizeof(uint64_t);
  hipEvent_t ev = take_event(s);
  if (!ev) return NTT_EDEVICE;
  if (hipMemcpyAsync(dst, s->base + r->out_off / sizeof(uint64_t), bytes, hipMemcpyDeviceToDevice,
                     (hipStream_t)stream) != hipSuccess ||
      hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
    // a copy that did reach the stream has run once this returns
    (void)hipStreamSynchronize((hipStream_t)stream);
    s->event_pool.push_back(ev);
    return NTT_EDEVICE;
  }
  r->read_events.push_back(ev);       // release frees the range only after this copy has run
  return NTT_OK;
}

ntt_status ntt_server_release(ntt_server* s, uint64_t ticket) {
  if (!s) return NTT_EINVAL_POINTER;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->records.find(ticket);
  if (it == s->records.end()) return NTT_ENOTFOUND;
  Req* r = it->second.get();
  if (r->state != NTT_REQ_DONE && r->state != NTT_REQ_FAILED) return NTT_EBUSY;
  if (r->has_out && !r->read_events.empty()) {
    // copies enqueued by ntt_server_read may not have run yet: the scheduler frees the
    // range once they have, so a request admitted into it cannot overwrite them
    PendingFree pf;
    pf.events.swap(r->read_events);
    pf.off[0] = r->out_off;
    pf.len[0] = r->out_len;
    r->has_out = false;
    s->pending_free.push_back(std::move(pf));
  } else {
    drop_out(s, r);
    for (hipEvent_t e : r->read_events) s->event_pool.push_back(e);
  }
  s->records.erase(it);
  s->cv_work.notify_one();
  return NTT_OK;
}

ntt_status ntt_server_stats_get(ntt_server* s, ntt_server_stats* out) {
  if (!s || !out) return NTT_EINVAL_POINTER;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  out->waiting = s->future.size() + s->ready.size();
  out->in_flight = s->outstanding - out->waiting;
  out->arena_bytes = s->arena.size();
  out->arena_in_use = s->arena.used();
  out->arena_peak = s->arena.peak();
  return NTT_OK;
}

ntt_status ntt_server_destroy(ntt_server* s) {
  if (!s) return NTT_EINVAL_POINTER;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->thread.joinable()) s->thread.join();
  destroy_resources(s);
  delete s;
  return NTT_OK;
}

}  // extern "C"
