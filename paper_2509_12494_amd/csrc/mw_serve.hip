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
//
// With config.resident, one- and two-word requests (up to resident_max_tiles
// tiles, by default every one the loop can take) instead go
// to the device-resident request loop (mw_resident.h): the scheduler (or the
// submitting thread, when the queue is empty) writes their descriptors into a
// ring in mapped host memory, a persistent kernel runs them, and the
// scheduler retires them by polling their done words there.  Both paths take
// requests from the one queue in arrival order and share the memory pool.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <array>
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
#include "mw_resident.h"
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
// A slot batch still running this long after its launch makes the resident
// loop yield (a slot batch of the serving mix takes tens of microseconds).
constexpr double kYieldAfterUs = 500.0;

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
  bool resident = false;   // runs in the device-resident loop
  uint64_t res_seq = 0;    // its entry number there
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
  double t_launch = 0;           // when its batch was launched
  std::vector<uint64_t> tickets;
};

bool is_ntt(uint32_t op) { return op <= MW_REQ_POLYMUL; }

// Host side of the device-resident loop (mw_resident.h).
struct Resident {
  ResHost* H = nullptr;          // mapped pinned block, host address
  ResHost* H_dev = nullptr;      // its device address
  ResDevBlock* D = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ended = nullptr;    // recorded after each launch
  bool launched = false;
  bool broken = false;           // a launch failed: resident requests fail
  uint32_t grid = 0;
  uint32_t route_tiles = kResRouteTiles;   // requests of at most this many tiles go to the loop
  uint64_t idle_ticks = 0, wait_ticks = 0, stall_ticks = 0;
  double last_query_us = 0;      // last check whether the loop has ended
  bool yielding = false;         // the yield word is set
  uint64_t published = 0;        // entries published
  uint64_t gpub = 0;             // tiles published
  uint64_t tiles_out = 0;        // tiles of published entries not yet complete
  std::vector<uint64_t> tile_start;     // per ring slot: global number of its entry's first tile
  std::vector<uint64_t> slot_ticket;    // per ring slot: ticket of its entry in flight, 0 if free
  std::vector<uint32_t> slot_tiles;
  std::vector<uint32_t> live;           // ring slots in flight
  // Barrett and Shoup constants of BLAS moduli, by (q, limbs)
  std::map<std::array<uint64_t, 3>, ModConst<4>> mod4;
  std::map<std::array<uint64_t, 3>, ModConst<2>> mod2;
  // tiles of a transform or product request, by (log2 N, limbs, job op)
  std::map<std::array<uint32_t, 3>, uint32_t> job_tiles;
};

// Tiles the batched executor splits a transform or product on `plan` into
// (they depend on N, the width and the operation only).
uint32_t ntt_tiles(Resident& X, ntt_plan_t plan, uint32_t log2n, uint32_t limbs, uint32_t op) {
  const std::array<uint32_t, 3> key = {log2n, limbs, op};
  auto it = X.job_tiles.find(key);
  if (it != X.job_tiles.end()) return it->second;
  if (it != X.job_tiles.end()) return it->second;
  ntt_job j;
  j.plan = plan;
  j.op = op;
  j.in = j.in2 = j.out = reinterpret_cast<void*>(kAlign);   // placeholders: nothing is read
  ExecPlan P;
  uint32_t tiles = UINT32_MAX;
  if (exec_build(&j, 1, P) == MW_OK) tiles = (uint32_t)P.items.size() + (uint32_t)P.items8.size();
  X.job_tiles.emplace(key, tiles);
  return tiles;
}

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
  Resident res;
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

// ---- device-resident loop ------------------------------------------------

// Fills ring entry E (number e) for an admitted request.  Status as mwntt.h.
int res_fill(mw_server_s* S, const Req& R, ResEntry& E, uint64_t e) {
  std::memset(&E, 0, sizeof(E));
  E.seq = e;
  if (is_ntt(R.r.op)) {
    ntt_job j;
    j.plan = R.r.plan;
    j.op = R.r.op == MW_REQ_NTT_FORWARD ? NTT_JOB_FORWARD
                                        : (R.r.op == MW_REQ_NTT_INVERSE ? NTT_JOB_INVERSE : NTT_JOB_POLYMUL);
    j.in = R.r.in;
    j.in2 = R.r.op == MW_REQ_POLYMUL ? R.r.in2 : nullptr;
    j.out = pool_ptr(S, R.out_off);
    ExecPlan plan;
    const int st = exec_build(&j, 1, plan);
    if (st != MW_OK) return st;
    JobDesc& d = plan.jobs[0];
    d.scratch = (u64)pool_ptr(S, R.scratch_off);
    uint32_t total = 0;
    for (u32 k = 0; k < d.nphases; ++k) {
      E.prefix[k] = total;
      total += d.tiles[k];
      if (plan.phase_lds[k] > kResLds) return MW_ESIZE;
    }
    if (total > kResMaxTiles || d.limbs > 2) return MW_ESIZE;
    E.prefix[d.nphases] = total;
    E.kind = RES_NTT;
    E.limbs = d.limbs;
    E.total = total;
    E.nphases = d.nphases;
    E.job = d;
    E.m4 = plan.m4[0];
    E.m2 = plan.m2[0];
    return MW_OK;
  }
  const uint32_t limbs = R.r.limbs;
  const uint64_t tiles = (R.r.n + kResBlasChunk - 1) / kResBlasChunk;
  if (limbs > 2 || tiles > kResMaxTiles) return MW_ESIZE;
  E.kind = RES_BLAS;
  E.limbs = limbs;
  E.total = (uint32_t)tiles;
  E.nphases = 1;
  E.prefix[1] = E.total;
  E.blas_op = R.r.op == MW_REQ_VEC_ADDMOD ? OP_ADD
              : R.r.op == MW_REQ_VEC_SUBMOD ? OP_SUB
              : R.r.op == MW_REQ_VEC_MULMOD ? OP_MUL : OP_AXPY;
  E.n = R.r.n;
  E.a = (u64)R.r.in;
  E.b = (u64)R.r.in2;
  E.c = (u64)pool_ptr(S, R.out_off);
  const std::array<uint64_t, 3> key = {R.r.q[0], limbs == 2 ? R.r.q[1] : 0, limbs};
  // a bounded memo: a stream of many distinct moduli starts it afresh
  if (S->res.mod4.size() + S->res.mod2.size() > 4096) {
    S->res.mod4.clear();
    S->res.mod2.clear();
  }
  if (limbs == 2) {
    auto it = S->res.mod4.find(key);
    if (it == S->res.mod4.end()) {
      ModConst<4> c = {};
      make_modulus<4>(R.r.q, 2, c.M);
      it = S->res.mod4.emplace(key, c).first;
    }
    E.m4 = it->second;
    if (E.blas_op == OP_AXPY && make_scalar<4>(R.r.alpha, R.r.q, 2, E.s4.w, E.s4.ws) != MW_OK) return MW_EINVAL;
  } else {
    auto it = S->res.mod2.find(key);
    if (it == S->res.mod2.end()) {
      ModConst<2> c = {};
      make_modulus<2>(R.r.q, 1, c.M);
      it = S->res.mod2.emplace(key, c).first;
    }
    E.m2 = it->second;
    if (E.blas_op == OP_AXPY && make_scalar<2>(R.r.alpha, R.r.q, 1, E.s2.w, E.s2.ws) != MW_OK) return MW_EINVAL;
  }
  return MW_OK;
}

void complete(mw_server_s* S, uint64_t tk, Req& R, bool failed) {
  R.state = failed ? RQ_FAILED : RQ_DONE;
  R.t_done = now_us();
  S->pool.release(R.scratch_off, R.scratch_bytes);
  R.scratch_bytes = 0;
  ++S->stats.completed;
  if (S->track_done) S->done_fifo.push_back(tk);
}

bool res_retire(mw_server_s* S);

// Fails the loop's entries in flight whose number is below `bound`.
void res_fail_live(mw_server_s* S, uint64_t bound) {
  Resident& X = S->res;
  for (size_t k = 0; k < X.live.size();) {
    const uint32_t slot = X.live[k];
    const uint64_t tk = X.slot_ticket[slot];
    Req& R = S->reqs[tk];
    if (R.res_seq >= bound) {
      ++k;
      continue;
    }
    complete(S, tk, R, true);
    X.tiles_out -= X.slot_tiles[slot];
    X.slot_ticket[slot] = 0;
    X.live[k] = X.live.back();
    X.live.pop_back();
  }
  S->cv_done.notify_all();
}

// Keeps the loop running while a published entry has not been taken: a loop
// that has ended is relaunched from the first entry it did not take.  With
// check_end it also looks whether the loop has ended with entries it took
// still incomplete (a stall bound ran out), and fails them.  false: a launch
// failed (the loop is marked broken).
bool res_ensure_running(mw_server_s* S, bool check_end) {
  Resident& X = S->res;
  uint64_t start = 0;
  if (X.launched) {
    start = __atomic_load_n(&X.H->consumed, __ATOMIC_ACQUIRE);
    const bool untaken = start < X.published;
    if (!untaken && !check_end) return true;
    X.last_query_us = now_us();
    if (hipEventQuery(X.ended) == hipErrorNotReady) return true;
    // the loop has ended: an entry it took and did not complete never will
    res_retire(S);
    res_fail_live(S, start);
    if (X.yielding) {
      __atomic_store_n(&X.H->yield, 0u, __ATOMIC_RELEASE);
      X.yielding = false;
    }
    if (!untaken) return true;
  }
  const uint64_t gstart = start < X.published ? X.tile_start[start & (kResRing - 1)] : X.gpub;
  ResCtl c = {};
  c.gcursor = gstart;
  c.completed = start;
  X.H->ctl_init = c;
  ResParams p;
  p.host = X.H_dev;
  p.dev = X.D;
  p.start_entry = start;
  p.gstart = gstart;
  p.idle_ticks = X.idle_ticks;
  p.wait_ticks = X.wait_ticks;
  p.stall_ticks = X.stall_ticks;
  // the per-slot counts start from zero: an entry failed by an ended loop
  // may have left its count part-way
  if (hipMemcpyAsync(&X.D->ctl, &X.H->ctl_init, sizeof(ResCtl), hipMemcpyHostToDevice, X.stream) != hipSuccess ||
      hipMemsetAsync(X.D->dcount, 0, sizeof(X.D->dcount) + sizeof(X.D->dfail) + sizeof(X.D->dphase), X.stream) != hipSuccess ||
      resident_launch(p, X.grid, X.stream) != hipSuccess || hipEventRecord(X.ended, X.stream) != hipSuccess) {
    X.broken = true;
    return false;
  }
  X.launched = true;
  ++S->stats.resident_launches;
  return true;
}

// Publishes the request at the head of the queue into the loop's ring.
// Returns false (and leaves it queued) when the ring, the tile ring or the
// memory budget has no room for it yet.
bool res_admit_head(mw_server_s* S) {
  Resident& X = S->res;
  const uint64_t tk = S->queue.front();
  Req& R = S->reqs[tk];
  const uint64_t e = X.published;
  const uint32_t slot = (uint32_t)(e & (kResRing - 1));
  if (X.broken) {
    // fails without having taken memory: nothing to return to the pool
    S->queue.pop_front();
    R.state = RQ_RUNNING;
    R.out_bytes = R.scratch_bytes = 0;
    complete(S, tk, R, true);
    S->cv_done.notify_all();
    return true;
  }
  if (X.slot_ticket[slot] || X.tiles_out + kResMaxTiles > kResTileRing) return false;
  size_t oo = 0, so = 0;
  if (!S->pool.alloc(R.out_bytes, &oo)) return false;
  if (!S->pool.alloc(R.scratch_bytes, &so)) {
    S->pool.release(oo, R.out_bytes);
    return false;
  }
  R.out_off = oo;
  R.scratch_off = so;
  R.state = RQ_RUNNING;
  S->queue.pop_front();
  S->stats.pool_peak = std::max(S->stats.pool_peak, S->pool.used());
  ResEntry& E = X.H->ring[slot];
  if (res_fill(S, R, E, e) != MW_OK) {
    complete(S, tk, R, true);
    S->cv_done.notify_all();
    return true;
  }
  R.res_seq = e;
  X.tile_start[slot] = X.gpub;
  X.gpub += E.total;
  X.tiles_out += E.total;
  X.slot_ticket[slot] = tk;
  X.slot_tiles[slot] = E.total;
  X.live.push_back(slot);
  X.published = e + 1;
  ++S->stats.resident_requests;
  __atomic_store_n(&X.H->tail, X.published, __ATOMIC_RELEASE);
  // the loop cannot run: nothing in flight will complete
  if (!res_ensure_running(S, false)) res_fail_live(S, UINT64_MAX);
  return true;
}

// Retires completed entries of the loop; true if any completed.
bool res_retire(mw_server_s* S) {
  Resident& X = S->res;
  bool any = false;
  for (size_t k = 0; k < X.live.size();) {
    const uint32_t slot = X.live[k];
    const uint64_t tk = X.slot_ticket[slot];
    Req& R = S->reqs[tk];
    const uint64_t d = __atomic_load_n(&X.H->done[slot], __ATOMIC_ACQUIRE);
    if ((d & ~(uint64_t(1) << 63)) != R.res_seq + 1) {
      ++k;
      continue;
    }
    complete(S, tk, R, (d >> 63) != 0);
    X.tiles_out -= X.slot_tiles[slot];
    X.slot_ticket[slot] = 0;
    X.live[k] = X.live.back();
    X.live.pop_back();
    any = true;
  }
  return any;
}

// Launches the run of slot-path requests at the head of the queue (up to
// max_batch, stopping at a request for the resident loop or one whose memory
// does not fit) on a free slot; false if nothing was launched.
bool admit_slot_batch(mw_server_s* S) {
  if (S->inflight >= S->cfg.max_inflight) return false;
  Slot* slot = nullptr;
  for (Slot& s : S->slots)
    if (!s.busy) {
      slot = &s;
      break;
    }
  if (!slot) return false;
  std::vector<uint64_t> batch;
  while (!S->queue.empty() && batch.size() < S->cfg.max_batch) {
    Req& R = S->reqs[S->queue.front()];
    if (R.resident) break;
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
  if (batch.empty()) return false;   // the oldest request waits for memory
  slot->busy = true;
  slot->t_launch = now_us();
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
    for (uint64_t tk : batch) complete(S, tk, S->reqs[tk], true);
    slot->tickets.clear();
    slot->busy = false;
    --S->inflight;
    S->cv_done.notify_all();
  }
  return true;
}

// Admits from the head of the queue: requests for the resident loop go into
// its ring, runs of other requests to a slot, in arrival order.
bool admit(mw_server_s* S) {
  bool progress = false;
  while (!S->queue.empty()) {
    const bool ok = S->reqs[S->queue.front()].resident ? res_admit_head(S) : admit_slot_batch(S);
    if (!ok) break;
    progress = true;
  }
  return progress;
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
      for (uint64_t tk : slot.tickets) complete(S, tk, S->reqs[tk], failed);
      slot.tickets.clear();
      slot.busy = false;
      --S->inflight;
      progress = true;
    }
    // a slot batch unfinished long after its launch may sit on the loop's
    // hardware queue behind the loop: ask the loop to yield (its entries
    // wait in the ring and the next launch takes them)
    if (S->res.launched && !S->res.yielding && S->inflight) {
      const double t = now_us();
      for (const Slot& slot : S->slots)
        if (slot.busy && t - slot.t_launch > kYieldAfterUs) {
          __atomic_store_n(&S->res.H->yield, 1u, __ATOMIC_RELEASE);
          S->res.yielding = true;
          ++S->stats.resident_yields;
          break;
        }
    }
    if (!S->res.live.empty()) {
      if (res_retire(S)) progress = true;
      // an entry published just as an idle loop left is taken by a new
      // launch; now and then, look whether the loop ended on a stall
      const size_t before = S->res.live.size();
      if (before) {
        const bool check_end = now_us() - S->res.last_query_us > 10000.0;
        if (!res_ensure_running(S, check_end)) res_fail_live(S, UINT64_MAX);
        if (S->res.live.size() != before) progress = true;
      }
    }
    if (progress) S->cv_done.notify_all();
    if (admit(S)) progress = true;
    const bool busy = S->inflight || !S->res.live.empty();
    if (S->stop && S->queue.empty() && !busy) break;
    if (progress) {
      last_action = now_us();
    } else if (S->cfg.spin_us && now_us() - last_action < S->cfg.spin_us) {
      // busy polling: let submitters take the lock, then look again
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      // poll completions often while work runs, otherwise sleep until work
      if (busy) S->cv_work.wait_for(lk, std::chrono::microseconds(4));
      else S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

int validate(mw_server_s* S, const mw_request& r, Req& R) {
  const uint32_t op = r.op;
  bool fits_resident = false;
  if (op > MW_REQ_VEC_AXPYMOD || !r.in) return MW_EINVAL;
  if (is_ntt(op)) {
    if (!r.plan) return MW_EINVAL;
    PlanView v;
    ModConst<8> c8;
    ModConst<4> c4;
    ModConst<2> c2;
    if (!plan_view(r.plan, v, c8, c4, c2) || v.variant) return MW_EINVAL;
    if (v.log2n < 6) return MW_ESIZE;
    fits_resident = S->cfg.resident && v.limbs <= 2 && v.log2n <= kResMaxLog2N &&
                    ntt_tiles(S->res, r.plan, v.log2n, v.limbs, op == MW_REQ_NTT_FORWARD ? NTT_JOB_FORWARD
                                              : (op == MW_REQ_NTT_INVERSE ? NTT_JOB_INVERSE : NTT_JOB_POLYMUL)) <=
                        S->res.route_tiles;
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
    fits_resident = r.limbs <= 2 && r.n <= (uint64_t)S->res.route_tiles * kResBlasChunk;
    R.cost_us = 1.0 + (double)R.out_bytes / 4.0e4;
  }
  if (R.out_bytes + R.scratch_bytes > S->pool.size()) return MW_ENOMEM;
  // the resident loop takes one- and two-word requests up to its tile limits;
  // validate mode checks inputs on a slot's stream, so it keeps the slot path
  if (S->cfg.resident && !S->cfg.dry_run && !validate_on()) {
    R.resident = fits_resident;
  }
  return MW_OK;
}

void free_server(mw_server_s* S) {
  for (Slot& s : S->slots) {
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.d_desc) (void)hipFree(s.d_desc);
    if (s.h_desc) (void)hipHostFree(s.h_desc);
  }
  Resident& X = S->res;
  if (X.stream) (void)hipStreamDestroy(X.stream);
  if (X.ended) (void)hipEventDestroy(X.ended);
  if (X.D) (void)hipFree(X.D);
  if (X.H) (void)hipHostFree(X.H);
  if (S->pool_base) (void)hipFree(S->pool_base);
  delete S;
}

// Memory, stream and clock constants of the resident loop (no launch yet:
// the first request launches it).
int init_resident(mw_server_s* S) {
  Resident& X = S->res;
  int cus = 0, khz = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S->device) != hipSuccess || cus <= 0 || khz <= 0)
    return MW_EDEVICE;
  // one worker per compute unit, plus the dispatcher (workgroup 0).  Two
  // per unit fit, but the tiles of a request then often share a unit, and a
  // phase lasts as long as its slowest tile: measured, the 2^17 two-word
  // transform took 52 us p50 with two workers per unit and 46 us with one.
  X.grid = (uint32_t)cus + 1;
  if (S->cfg.resident_max_tiles) X.route_tiles = S->cfg.resident_max_tiles;
  X.idle_ticks = (uint64_t)khz * 20;      // 20 ms
  X.wait_ticks = S->cfg.resident_wait_us ? (uint64_t)khz * S->cfg.resident_wait_us / 1000
                                         : (uint64_t)khz * 2000;   // 2 s
  X.stall_ticks = (uint64_t)khz * 5000;   // 5 s
  X.tile_start.assign(kResRing, 0);
  X.slot_ticket.assign(kResRing, 0);
  X.slot_tiles.assign(kResRing, 0);
  if (hipHostMalloc(reinterpret_cast<void**>(&X.H), sizeof(ResHost), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&X.D), sizeof(ResDevBlock)) != hipSuccess)
    return MW_ENOMEM;
  std::memset(X.H, 0, sizeof(ResHost));
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&X.H_dev), X.H, 0) != hipSuccess ||
      hipMemset(X.D, 0, sizeof(ResDevBlock)) != hipSuccess ||
      // no tile word may carry a valid tag before the dispatcher writes it
      hipMemset(X.D->tiles, 0xff, sizeof(X.D->tiles)) != hipSuccess ||
      hipStreamCreateWithFlags(&X.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&X.ended, hipEventDisableTiming) != hipSuccess)
    return MW_EDEVICE;
  return MW_OK;
}

}  // namespace

extern "C" int mw_server_create(mw_server_t* out, const mw_server_config* cfg) {
  if (!out || !cfg) return MW_EINVAL;
  *out = nullptr;
  if (cfg->max_inflight < 1 || cfg->max_inflight > 16 || cfg->max_batch < 1 || cfg->max_batch > kMaxBatch ||
      cfg->hbm_budget < kAlign || cfg->spin_us > 100000 || cfg->resident_max_tiles > kResMaxTiles)
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
    if (st == MW_OK && cfg->resident) st = init_resident(S);
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
  // a request for the resident loop that finds the queue empty is published
  // by the submitting thread itself, without waiting for the scheduler
  if (S->queue.size() == 1 && S->reqs[t].resident) res_admit_head(S);
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
  if (S->res.launched) {
    // every request has completed: the loop leaves at its next look
    __atomic_store_n(&S->res.H->stop, 1u, __ATOMIC_RELEASE);
    (void)hipStreamSynchronize(S->res.stream);
  }
  if (!S->cfg.dry_run) (void)hipDeviceSynchronize();
  free_server(S);
  return MW_OK;
}
