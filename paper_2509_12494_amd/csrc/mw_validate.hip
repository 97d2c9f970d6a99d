// Validate mode (see mw_set_validate in mwntt.h): a streaming check kernel
// that compares every input residue with q and records a violation in one
// library-wide error word.  The word lives in pinned host memory so that the
// host can read it after the check has completed without a device copy;
// every writer stores the same value, so no atomic is needed.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "mw_arith.h"
#include "mw_common.h"
#include "mw_validate.h"

namespace mw {

template <int W>
struct QWords {
  u32 q[W];
};

// Grid-stride over the residues; lane i sets *err when any of its residues is
// >= q (the borrow of x - q is clear).
template <int W>
__global__ __launch_bounds__(256) void canon_check_kernel(const Res<W>* x, u64 n, QWords<W> Q, u32* err) {
  bool bad = false;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
    u32 borrow;
    (void)sub(ResIO<W>::load(x + i), Q.q, borrow);
    bad |= borrow == 0;
  }
  if (bad) *err = 1u;
}

namespace {
std::mutex g_mu;
std::atomic<int> g_on{-1};                 // -1: not yet read from the environment
std::atomic<uint32_t*> g_word{nullptr};    // pinned host word, device-visible

// Allocates the error word once (pinned, mapped into the device address space).
uint32_t* error_word() {
  uint32_t* w = g_word.load(std::memory_order_acquire);
  if (w) return w;
  std::lock_guard<std::mutex> lk(g_mu);
  w = g_word.load(std::memory_order_relaxed);
  if (w) return w;
  void* p = nullptr;
  if (hipHostMalloc(&p, 256, hipHostMallocMapped | hipHostMallocPortable) != hipSuccess) return nullptr;
  std::memset(p, 0, 256);
  w = static_cast<uint32_t*>(p);
  g_word.store(w, std::memory_order_release);
  return w;
}

int set_on(bool on) {
  if (on && !error_word()) return MW_ENOMEM;
  g_on.store(on ? 1 : 0, std::memory_order_release);
  return MW_OK;
}

template <int W>
int launch_check(const void* d_x, uint64_t count, const uint64_t* q, uint32_t limbs, hipStream_t s, uint32_t* err) {
  QWords<W> Q{};
  for (int i = 0; i < W; ++i) Q.q[i] = (u32)(q[i / 2] >> (32 * (i % 2)));
  (void)limbs;
  const u64 blocks = (count + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
  void* dev_err = nullptr;
  if (hipHostGetDevicePointer(&dev_err, err, 0) != hipSuccess) return MW_EDEVICE;
  hipLaunchKernelGGL((canon_check_kernel<W>), dim3(grid), dim3(256), 0, s, reinterpret_cast<const Res<W>*>(d_x),
                     (u64)count, Q, static_cast<u32*>(dev_err));
  return hipGetLastError() == hipSuccess ? MW_OK : MW_EDEVICE;
}
}  // namespace

bool validate_on() {
  int on = g_on.load(std::memory_order_acquire);
  if (on < 0) {
    const char* env = std::getenv("MWNTT_VALIDATE");
    const bool want = env && env[0] && std::strcmp(env, "0") != 0;
    if (set_on(want) != MW_OK) g_on.store(0, std::memory_order_release);
    on = g_on.load(std::memory_order_acquire);
  }
  return on > 0;
}

int validate_take() {
  uint32_t* w = g_word.load(std::memory_order_acquire);
  if (!w) return MW_OK;
  if (__atomic_exchange_n(w, 0u, __ATOMIC_ACQ_REL) != 0u) return MW_ENONCANON;
  return MW_OK;
}

int validate_input(const void* d_x, uint64_t count, const uint64_t* q, uint32_t limbs, hipStream_t s) {
  if (!validate_on() || count == 0) return MW_OK;
  uint32_t* err = error_word();
  if (!err) return MW_ENOMEM;
  switch (limbs) {
    case 4: return launch_check<8>(d_x, count, q, limbs, s, err);
    case 2: return launch_check<4>(d_x, count, q, limbs, s, err);
    default: return launch_check<2>(d_x, count, q, limbs, s, err);
  }
}

}  // namespace mw

extern "C" int mw_set_validate(int on) {
  (void)mw::validate_on();   // settle the environment default first
  return mw::set_on(on != 0);
}

extern "C" int mw_get_validate(void) { return mw::validate_on() ? 1 : 0; }

extern "C" int mw_check(void* stream) {
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return MW_EDEVICE;
  return mw::validate_take();
}
