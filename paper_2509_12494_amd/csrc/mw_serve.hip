// Serving runtime: continuous batching of NTT / modular BLAS requests with
// HBM-budget admission (see the mw_server_* section of mwntt.h).
//
// State: a FIFO of queued requests, a first-fit pool over one device
// allocation of `hbm_budget` bytes (outputs and scratch of admitted
// requests), and `max_inflight` slots, each a stream with an event and
// preallocated descriptor buffers (device + pinned host staging).  A
// scheduler thread loops: it retires slots whose event completed (their
// requests become complete and their scratch returns to the pool), then, while
// a slot is free, admits requests from the head of the queue as long as their
// memory fits and the batch has room, uploads the batch's descriptors with
// one asynchronous copy (a batch of one transform or product passes its
// descriptor in the kernel arguments instead, with no copy) and launches it (transform / product requests through
// the batched executor, BLAS requests as their own kernels) on the slot's
// stream.  Requests arriving meanwhile wait in the queue and go into the next
// batch on the next free slot, so batches overlap on the device.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mw_common.h"
#include "mw_exec.h"
#include "mw_validate.h"

namespace mw {
int blas_launch(int op, void* d_c, const void* d_a, const void* d_b, size_t n, const uint64_t* q, uint32_t limbs,
                const uint64_t* alpha, void* stream);
}

using namespace mw;

namespace {

constexpr size_t kAlign = 256;
constexpr uint32_t kMaxBatch = 256;
constexpr uint32_t kMaxTilesPerJob = 2048;

double now_us() {
  using namespace std::chrono;
  return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

size_t round_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Pool {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = peak_ = 0;
  }
  // returns false if no free block is large enough
  bool alloc(size_t bytes, size_t* off) {
    if (bytes == 0) {
      *off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    if (bytes == 0) return;
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    size_t start = off, len = bytes;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + bytes == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0, peak_ = 0;
};

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_DONE, RQ_FAILED };

// Byte offsets of the parts of a packed descriptor block, each 256-byte aligned.
struct DescLayout {
  size_t jobs = 0, m8 = 0, m4 = 0, m2 = 0, items = 0, items8 = 0, total = 0;
};
DescLayout desc_layout(size_t nj, size_t ni, size_t ni8) {
  auto up = [](size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); };
  DescLayout L;
  L.m8 = up(sizeof(JobDesc) * nj);
  L.m4 = L.m8 + up(sizeof(ModConst<8>) * nj);
  L.m2 = L.m4 + up(sizeof(ModConst<4>) * nj);
  L.items = L.m2 + up(sizeof(ModConst<2>) * nj);
  L.items8 = L.items + up(sizeof(uint2) * ni);
  L.total = L.items8 + sizeof(uint2) * ni8;
  return L;
}

struct Req {
  mw_request r;
  size_t out_bytes = 0, scratch_bytes = 0;
  size_t out_off = 0, scratch_off = 0;
  double t_submit = 0, t_done = 0;
  double cost_us = 0;   // dry-run model
  ReqState state = RQ_QUEUED;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  // A batch's descriptors (jobs, per-job constants, tile lists) packed into
  // one block, staged in pinned memory and sent with a single copy.
  char* d_desc = nullptr;
  char* h_desc = nullptr;
  bool busy = false;
  double t_end = 0;              // dry run
  std::vector<uint64_t> tickets;
};

bool is_ntt(uint32_t op) { return op <= MW_REQ_POLYMUL; }

}  // namespace

struct mw_server_s {
  mw_server_config cfg{};
  int device = 0;
  void* pool_base = nullptr;
  Pool pool;
  std::vector<Slot> slots;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;
  uint64_t next_ticket = 1;
  uint32_t inflight = 0;
  mw_server_stats stats{};
  bool stop = false;
  // completion log for mw_server_replay: while `track_done` is set the
  // scheduler appends every completed ticket
  bool track_done = false;
  std::deque<uint64_t> done_fifo;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread sched;
};

namespace {

void* pool_ptr(mw_server_s* S, size_t off) { return S->pool_base ? (char*)S->pool_base + off : nullptr; }

// Several transforms / products: descriptors packed into the slot's pinned
// block, sent with one copy, then the executor's launches.
bool launch_packed(Slot& slot, const ExecPlan& plan) {
  const size_t nj = plan.jobs.size(), ni = plan.items.size(), ni8 = plan.items8.size();
  const DescLayout L = desc_layout(nj, ni, ni8);
  std::memcpy(slot.h_desc + L.jobs, plan.jobs.data(), sizeof(JobDesc) * nj);
  std::memcpy(slot.h_desc + L.m8, plan.m8.data(), sizeof(ModConst<8>) * nj);
  std::memcpy(slot.h_desc + L.m4, plan.m4.data(), sizeof(ModConst<4>) * nj);
  std::memcpy(slot.h_desc + L.m2, plan.m2.data(), sizeof(ModConst<2>) * nj);
  std::memcpy(slot.h_desc + L.items, plan.items.data(), sizeof(uint2) * ni);
  std::memcpy(slot.h_desc + L.items8, plan.items8.data(), sizeof(uint2) * ni8);
  if (hipMemcpyAsync(slot.d_desc, slot.h_desc, L.total, hipMemcpyHostToDevice, slot.stream) != hipSuccess)
    return false;
  char* b = slot.d_desc;
  const ExecDevice d{(const JobDesc*)(b + L.jobs), (const uint2*)(b + L.items), (const uint2*)(b + L.items8),
                     (const ModConst<8>*)(b + L.m8), (const ModConst<4>*)(b + L.m4),
                     (const ModConst<2>*)(b + L.m2)};
  return exec_launch(d, plan, slot.stream) == hipSuccess;
}

// Launch one batch on a slot (called with the lock held).
bool launch_batch(mw_server_s* S, Slot& slot, const std::vector<uint64_t>& batch) {
  slot.tickets = batch;
  if (S->cfg.dry_run) {
    double cost = 5.0;
    for (uint64_t t : batch) cost += S->reqs[t].cost_us;
    slot.t_end = now_us() + cost;
    return true;
  }
  std::vector<ntt_job> jobs;
  std::vector<uint64_t> job_tickets;
  for (uint64_t t : batch) {
    Req& R = S->reqs[t];
    if (!is_ntt(R.r.op)) continue;
    ntt_job j;
    j.plan = R.r.plan;
    j.op = R.r.op == MW_REQ_NTT_FORWARD ? NTT_JOB_FORWARD
                                        : (R.r.op == MW_REQ_NTT_INVERSE ? NTT_JOB_INVERSE : NTT_JOB_POLYMUL);
    j.in = R.r.in;
    j.in2 = R.r.op == MW_REQ_POLYMUL ? R.r.in2 : nullptr;
    j.out = pool_ptr(S, R.out_off);
    jobs.push_back(j);
    job_tickets.push_back(t);
  }
  if (!jobs.empty()) {
    ExecPlan plan;
    if (exec_build(jobs.data(), (uint32_t)jobs.size(), plan) != MW_OK) return false;
    if (plan.items.size() > (size_t)S->cfg.max_batch * kMaxTilesPerJob ||
        plan.items8.size() > (size_t)S->cfg.max_batch * kMaxTilesPerJob)
      return false;
    for (size_t i = 0; i < jobs.size(); ++i) plan.jobs[i].scratch = (u64)pool_ptr(S, S->reqs[job_tickets[i]].scratch_off);
    if (exec_prepare(plan) != hipSuccess) return false;
    if (validate_on() && exec_validate(plan, slot.stream) != MW_OK) return false;
    if (jobs.size() == 1) {
      // one transform or product: its descriptor goes in the kernel arguments
      if (exec_launch_one(plan, slot.stream) != hipSuccess) return false;
    } else if (!launch_packed(slot, plan)) {
      return false;
    }
  }
  for (uint64_t t : batch) {
    Req& R = S->reqs[t];
    if (is_ntt(R.r.op)) continue;
    const int op = R.r.op == MW_REQ_VEC_ADDMOD ? 0 : R.r.op == MW_REQ_VEC_SUBMOD ? 1 : R.r.op == MW_REQ_VEC_MULMOD ? 2 : 3;
    if (blas_launch(op, pool_ptr(S, R.out_off), R.r.in, R.r.in2, R.r.n, R.r.q, R.r.limbs, R.r.alpha, slot.stream) !=
        MW_OK)
      return false;
  }
  return hipEventRecord(slot.done, slot.stream) == hipSuccess;
}

void scheduler(mw_server_s* S) {
  if (!S->cfg.dry_run) (void)hipSetDevice(S->device);
  // While batches run the loop re-checks their events every few microseconds
  // with a timed wait; Linux lets a timed wait overrun by the thread's timer
  // slack (50 us by default), which would add that much to every request's
  // latency.  1 us of slack keeps the polling interval what it says.
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  std::unique_lock<std::mutex> lk(S->mu);
  double last_action = now_us();
  for (;;) {
    bool progress = false;
    // retire finished batches
    for (Slot& slot : S->slots) {
      if (!slot.busy) continue;
      bool done, failed = false;
      if (S->cfg.dry_run) {
        done = now_us() >= slot.t_end;
      } else {
        const hipError_t e = hipEventQuery(slot.done);
        done = e != hipErrorNotReady;
        failed = done && e != hipSuccess;
      }
      if (!done) continue;
      const double t = now_us();
      for (uint64_t tk : slot.tickets) {
        Req& R = S->reqs[tk];
        R.state = failed ? RQ_FAILED : RQ_DONE;
        R.t_done = t;
        S->pool.release(R.scratch_off, R.scratch_bytes);
        R.scratch_bytes = 0;
        ++S->stats.completed;
        if (S->track_done) S->done_fifo.push_back(tk);
      }
      slot.tickets.clear();
      slot.busy = false;
      --S->inflight;
      progress = true;
    }
    if (progress) S->cv_done.notify_all();
    // admit and launch
    while (S->inflight < S->cfg.max_inflight && !S->queue.empty()) {
      Slot* slot = nullptr;
      for (Slot& s : S->slots)
        if (!s.busy) {
          slot = &s;
          break;
        }
      if (!slot) break;
      std::vector<uint64_t> batch;
      while (!S->queue.empty() && batch.size() < S->cfg.max_batch) {
        Req& R = S->reqs[S->queue.front()];
        size_t oo = 0, so = 0;
        if (!S->pool.alloc(R.out_bytes, &oo)) break;
        if (!S->pool.alloc(R.scratch_bytes, &so)) {
          S->pool.release(oo, R.out_bytes);
          break;
        }
        R.out_off = oo;
        R.scratch_off = so;
        R.state = RQ_RUNNING;
        batch.push_back(S->queue.front());
        S->queue.pop_front();
      }
      if (batch.empty()) break;   // the oldest request waits for memory
      slot->busy = true;
      ++S->inflight;
      ++S->stats.batches;
      S->stats.max_batch_seen = std::max<uint64_t>(S->stats.max_batch_seen, batch.size());
      S->stats.inflight_peak = std::max<uint64_t>(S->stats.inflight_peak, S->inflight);
      S->stats.pool_peak = std::max(S->stats.pool_peak, S->pool.used());
      if (!launch_batch(S, *slot, batch)) {
        // the batch could not be launched: part of it may already be queued on
        // the slot's stream (kernels, the descriptor copy from the slot's
        // pinned block), so wait for the stream before its scratch, outputs
        // and pinned block are reused; then fail its requests, free the slot
        if (!S->cfg.dry_run) (void)hipStreamSynchronize(slot->stream);
        for (uint64_t tk : batch) {
          Req& R = S->reqs[tk];
          R.state = RQ_FAILED;
          R.t_done = now_us();
          S->pool.release(R.scratch_off, R.scratch_bytes);
          R.scratch_bytes = 0;
          ++S->stats.completed;
          if (S->track_done) S->done_fifo.push_back(tk);
        }
        slot->tickets.clear();
        slot->busy = false;
        --S->inflight;
        S->cv_done.notify_all();
      }
      progress = true;
    }
    if (S->stop && S->queue.empty() && S->inflight == 0) break;
    if (progress) {
      last_action = now_us();
    } else if (S->cfg.spin_us && now_us() - last_action < S->cfg.spin_us) {
      // busy polling: let submitters take the lock, then look again
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      // poll completions often while batches run, otherwise sleep until work
      if (S->inflight) S->cv_work.wait_for(lk, std::chrono::microseconds(4));
      else S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

int validate(mw_server_s* S, const mw_request& r, Req& R) {
  const uint32_t op = r.op;
  if (op > MW_REQ_VEC_AXPYMOD || !r.in) return MW_EINVAL;
  if (is_ntt(op)) {
    if (!r.plan) return MW_EINVAL;
    PlanView v;
    ModConst<8> c8;
    ModConst<4> c4;
    ModConst<2> c2;
    if (!plan_view(r.plan, v, c8, c4, c2) || v.variant) return MW_EINVAL;
    if (v.log2n < 6) return MW_ESIZE;
    if (op == MW_REQ_POLYMUL) {
      if (!r.in2) return MW_EINVAL;
      if (check_modulus(v.q, v.limbs) != MW_OK) return MW_EMODULUS;
    }
    const size_t bytes = (size_t)8 * v.limbs << v.log2n;
    R.out_bytes = round_up(bytes);
    R.scratch_bytes = round_up((op == MW_REQ_POLYMUL ? 2 : 1) * bytes);
    R.cost_us = 1.0 + (double)bytes * v.log2n / 8.0e4;
  } else {
    if (!r.in2 || r.n == 0) return MW_EINVAL;
    if (r.n > (uint64_t(1) << 40)) return MW_EINVAL;   // the BLAS length limit; keeps 8*limbs*n exact
    int st = check_modulus(r.q, r.limbs);
    if (st != MW_OK) return st;
    if (op == MW_REQ_VEC_AXPYMOD) {
      const mwhost::U256 Q = mwhost::u256_from_words(r.q, r.limbs), A = mwhost::u256_from_words(r.alpha, r.limbs);
      if (!(A < Q)) return MW_EINVAL;
    }
    R.out_bytes = round_up((size_t)8 * r.limbs * r.n);
    R.scratch_bytes = 0;
    R.cost_us = 1.0 + (double)R.out_bytes / 4.0e4;
  }
  if (R.out_bytes + R.scratch_bytes > S->pool.size()) return MW_ENOMEM;
  return MW_OK;
}

void free_server(mw_server_s* S) {
  for (Slot& s : S->slots) {
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.d_desc) (void)hipFree(s.d_desc);
    if (s.h_desc) (void)hipHostFree(s.h_desc);
  }
  if (S->pool_base) (void)hipFree(S->pool_base);
  delete S;
}

}  // namespace

extern "C" int mw_server_create(mw_server_t* out, const mw_server_config* cfg) {
  if (!out || !cfg) return MW_EINVAL;
  *out = nullptr;
  if (cfg->max_inflight < 1 || cfg->max_inflight > 16 || cfg->max_batch < 1 || cfg->max_batch > kMaxBatch ||
      cfg->hbm_budget < kAlign || cfg->spin_us > 100000)
    return MW_EINVAL;
  mw_server_s* S = new (std::nothrow) mw_server_s();
  if (!S) return MW_ENOMEM;
  S->cfg = *cfg;
  S->pool.init(cfg->hbm_budget & ~(kAlign - 1));
  S->slots.resize(cfg->max_inflight);
  if (!cfg->dry_run) {
    int st = MW_OK;
    if (hipGetDevice(&S->device) != hipSuccess) st = MW_EDEVICE;
    if (st == MW_OK && hipMalloc(&S->pool_base, S->pool.size()) != hipSuccess) st = MW_ENOMEM;
    const size_t ni = (size_t)cfg->max_batch * kMaxTilesPerJob;
    const size_t cap = desc_layout(cfg->max_batch, ni, ni).total;
    for (Slot& s : S->slots) {
      if (st != MW_OK) break;
      if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
        st = MW_EDEVICE;
        break;
      }
      if (hipMalloc(&s.d_desc, cap) != hipSuccess || hipHostMalloc(&s.h_desc, cap) != hipSuccess)
        st = MW_ENOMEM;
    }
    if (st != MW_OK) {
      free_server(S);
      return st;
    }
  }
  try {
    S->sched = std::thread(scheduler, S);
  } catch (...) {
    free_server(S);
    return MW_ENOMEM;
  }
  *out = S;
  return MW_OK;
}

namespace {
// Queue a request; the caller holds S->mu.
int submit_locked(mw_server_s* S, const mw_request* request, uint64_t* ticket) {
  Req R;
  R.r = *request;
  int st = validate(S, *request, R);
  if (st != MW_OK) return st;
  R.t_submit = now_us();
  const uint64_t t = S->next_ticket++;
  S->reqs.emplace(t, R);
  S->queue.push_back(t);
  ++S->stats.submitted;
  S->stats.queue_peak = std::max<uint64_t>(S->stats.queue_peak, S->queue.size());
  *ticket = t;
  S->cv_work.notify_one();
  return MW_OK;
}
}  // namespace

extern "C" int mw_server_submit(mw_server_t S, const mw_request* request, uint64_t* ticket) {
  if (!S || !request || !ticket) return MW_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  return submit_locked(S, request, ticket);
}

extern "C" int mw_server_result(mw_server_t S, uint64_t ticket, int wait, void** d_out, double* latency_us) {
  if (!S) return MW_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return MW_EINVAL;
  if (wait) {
    // the entry can be erased meanwhile (mw_server_release on another thread,
    // or replay's collector): look it up by find() so a wait never inserts one
    S->cv_done.wait(lk, [&] {
      const auto f = S->reqs.find(ticket);
      return f == S->reqs.end() || f->second.state == RQ_DONE || f->second.state == RQ_FAILED;
    });
    it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return MW_EINVAL;
  }
  Req& R = it->second;
  if (R.state == RQ_QUEUED || R.state == RQ_RUNNING) return MW_EBUSY;
  if (R.state == RQ_FAILED) return MW_EDEVICE;
  if (d_out) *d_out = pool_ptr(S, R.out_off);
  if (latency_us) *latency_us = R.t_done - R.t_submit;
  return MW_OK;
}

extern "C" int mw_server_release(mw_server_t S, uint64_t ticket) {
  if (!S) return MW_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return MW_EINVAL;
  if (it->second.state == RQ_QUEUED || it->second.state == RQ_RUNNING) return MW_EBUSY;
  S->pool.release(it->second.out_off, it->second.out_bytes);
  S->reqs.erase(it);
  S->cv_work.notify_one();
  return MW_OK;
}

extern "C" int mw_server_drain(mw_server_t S) {
  if (!S) return MW_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return S->queue.empty() && S->inflight == 0; });
  return MW_OK;
}

extern "C" int mw_server_get_stats(mw_server_t S, mw_server_stats* stats) {
  if (!S || !stats) return MW_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  *stats = S->stats;
  stats->pool_peak = S->pool.peak();
  return MW_OK;
}

extern "C" int mw_server_replay(mw_server_t S, const mw_request* reqs, const double* arrival_us, uint32_t count,
                                double* latency_us, double* makespan_us) {
  if (!S || !reqs || !arrival_us || !latency_us || count == 0) return MW_EINVAL;
  std::unordered_map<uint64_t, uint32_t> index;   // ticket -> request position
  index.reserve(count * 2);
  int status = MW_OK;
  uint32_t done = 0;
  const double t0 = now_us();
  double last_done = t0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->track_done) return MW_EBUSY;            // one replay at a time
    S->track_done = true;
    S->done_fifo.clear();
  }
  // collector: releases each completed request as the scheduler reports it
  std::thread collector([&] {
    std::unique_lock<std::mutex> lk(S->mu);
    while (done < count) {
      if (S->done_fifo.empty()) {
        S->cv_done.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
      while (!S->done_fifo.empty()) {
        const uint64_t tk = S->done_fifo.front();
        S->done_fifo.pop_front();
        auto pos = index.find(tk);
        auto it = S->reqs.find(tk);
        if (pos == index.end() || it == S->reqs.end()) continue;   // not part of this replay
        Req& R = it->second;
        if (R.state == RQ_FAILED) status = MW_EDEVICE;
        latency_us[pos->second] = R.t_done - (t0 + arrival_us[pos->second]);
        last_done = std::max(last_done, R.t_done);
        S->pool.release(R.out_off, R.out_bytes);
        S->reqs.erase(it);
        ++done;
      }
      S->cv_work.notify_one();
    }
  });
  for (uint32_t i = 0; i < count; ++i) {
    const double target = t0 + arrival_us[i];
    for (;;) {
      const double d = target - now_us();
      if (d <= 0) break;
      if (d > 200) std::this_thread::sleep_for(std::chrono::microseconds((long)(d - 100)));
    }
    std::lock_guard<std::mutex> lk(S->mu);
    uint64_t tk = 0;
    const int st = submit_locked(S, &reqs[i], &tk);
    if (st == MW_OK) {
      index.emplace(tk, i);
    } else {
      // rejected requests count as failed and complete at once
      status = st;
      latency_us[i] = 0;
      ++done;
      S->cv_done.notify_all();
    }
  }
  collector.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->track_done = false;
    S->done_fifo.clear();
  }
  if (makespan_us) *makespan_us = last_done - t0;
  return status;
}

extern "C" int mw_server_destroy(mw_server_t S) {
  if (!S) return MW_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->sched.joinable()) S->sched.join();
  if (!S->cfg.dry_run) (void)hipDeviceSynchronize();
  free_server(S);
  return MW_OK;
}
