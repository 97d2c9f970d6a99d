// The serving runtime's device-resident request loop (protocol in
// mw_resident.h): a dispatcher workgroup moving published requests from the
// mapped host ring into device memory and the tile ring, and worker
// workgroups running the tiles -- transform and product tiles through the
// batched executor's tile bodies (run-time line engine), BLAS tiles as
// chunks of element-wise operations.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "mw_exec_tiles.h"
#include "mw_resident.h"

namespace mw {

namespace {

constexpr u32 kEntryUnits = sizeof(ResEntry) / 16;
// the 16-byte unit of a descriptor whose first word is its tile count
constexpr u32 kTotalUnit = offsetof(ResEntry, total) / 16;
static_assert(offsetof(ResEntry, total) % 16 == 0, "the tile count starts a 16-byte unit");

__device__ __forceinline__ void fence_acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T load_system(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every wave waits until its own memory operations have completed (stores
// acknowledged by the L2), so that one wave's release afterwards covers the
// whole workgroup's stores.  (A workgroup barrier does not wait for them.)
__device__ __forceinline__ void wait_own_stores() { __builtin_amdgcn_s_waitcnt(0); }

// 16-byte copy of a descriptor by the workgroup's lanes.
__device__ __forceinline__ void copy_entry(ResEntry* dst, const ResEntry* src) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  for (u32 k = threadIdx.x; k < kEntryUnits; k += blockDim.x) d[k] = s[k];
}

__device__ __forceinline__ void dispatch(const ResParams& p, u64& sh_a, u32& sh_b) {
  ResHost* H = p.host;
  ResDevBlock* D = p.dev;
  const u32 t = threadIdx.x;
  u64 consumed = p.start_entry, gpub = p.gstart;
  // lane 0 keeps the clocks and takes every decision; the workgroup follows
  // its flags, so all lanes leave the loop at the same iteration
  u64 last = wall_clock64();          // last entry taken
  u64 progress = last;                // last entry taken or completed
  u64 seen_done = p.start_entry;
  u32 beat = 0;
  for (;;) {
    if (t == 0) {
      store_agent(&D->ctl.beat, ++beat);
      // while the host asks to yield, no new entry is taken; the three words
      // are read together (one PCIe round trip)
      const u32 yielding = load_system(&H->yield);
      const u64 tail = load_system(&H->tail);
      const u32 stop = load_system(&H->stop) | yielding;
      sh_a = yielding ? consumed : tail;
      const u64 done = load_agent(&D->ctl.completed);
      const u64 now = wall_clock64();
      if (done != seen_done) {
        seen_done = done;
        progress = now;
      }
      // 1: the host asks to stop, 2: every entry taken is complete,
      // 4: entries are pending but none completed for the stall bound,
      // 8: no entry arrived for the idle time
      sh_b = (stop ? 1u : 0u) | (done == consumed ? 2u : 0u) | (now - progress > p.stall_ticks ? 4u : 0u) |
             (now - last > p.idle_ticks ? 8u : 0u);
    }
    __syncthreads();
    const u64 tail = sh_a;
    const u32 flags = sh_b;
    __syncthreads();
    if (tail > consumed) {
      // the host wrote the entries before it stored tail
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
      for (; consumed < tail; ++consumed) {
        const u32 slot = (u32)(consumed & (kResRing - 1));
        {
          // one PCIe round trip: each lane moves 16-byte units, and the lane
          // holding the unit with the tile count passes it on through LDS
          const uint4* src = reinterpret_cast<const uint4*>(&H->ring[slot]);
          uint4* dst = reinterpret_cast<uint4*>(&D->dent[slot]);
          for (u32 k = t; k < kEntryUnits; k += blockDim.x) {
            const uint4 u = src[k];
            dst[k] = u;
            if (k == kTotalUnit) sh_b = u.x;
          }
        }
        // the descriptor is visible at agent scope before any tile word of it
        wait_own_stores();
        __syncthreads();
        const u32 total = sh_b;
        fence_release_agent();
        for (u32 i = t; i < total; i += blockDim.x) {
          const u64 g = gpub + i;
          store_agent(&D->tiles[g & (kResTileRing - 1)], ((g & kResTagMask) << 24) | ((u64)slot << 12) | i);
        }
        gpub += total;
        __syncthreads();   // every lane has read the count before the next entry's is written
      }
      if (t == 0) {
        __hip_atomic_store(&H->consumed, consumed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        last = progress = wall_clock64();
      }
      continue;
    }
    if ((flags & 2) && (flags & (1u | 8u))) break;
    if (flags & 4) {
      if (t == 0) store_agent(&D->ctl.error, 2u);
      break;
    }
    __builtin_amdgcn_s_sleep(16);
  }
  if (t == 0) __hip_atomic_store(&D->ctl.stop, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W, int OP, bool NORM>
__device__ __forceinline__ void blas_tile_op(const ResEntry& E, const Modulus<W>& M, const Scalar<W>& s, u32 tile) {
  const Res<W>* a = reinterpret_cast<const Res<W>*>(E.a);
  const Res<W>* b = reinterpret_cast<const Res<W>*>(E.b);
  Res<W>* c = reinterpret_cast<Res<W>*>(E.c);
  const u64 lo = (u64)tile * kResBlasChunk;
  const u64 hi = lo + kResBlasChunk < E.n ? lo + kResBlasChunk : E.n;
  for (u64 i = lo + threadIdx.x; i < hi; i += blockDim.x)
    LoopIO::store(c + i, blas_elem<W, OP, NORM>(ResIO<W>::load(a + i), ResIO<W>::load(b + i), M, s));
}

template <int W>
__device__ __forceinline__ void blas_tile(const ResEntry& E, const ModConst<W>& mc, const Scalar<W>& s, u32 tile) {
  switch (E.blas_op) {
    case OP_ADD: blas_tile_op<W, OP_ADD, false>(E, mc.M, s, tile); break;
    case OP_SUB: blas_tile_op<W, OP_SUB, false>(E, mc.M, s, tile); break;
    case OP_MUL:
      if (mc.M.shift) blas_tile_op<W, OP_MUL, true>(E, mc.M, s, tile);
      else blas_tile_op<W, OP_MUL, false>(E, mc.M, s, tile);
      break;
    default: blas_tile_op<W, OP_AXPY, false>(E, mc.M, s, tile); break;
  }
}

__device__ __forceinline__ void work(const ResParams& p, ResEntry& E, u64& sh_word, u32& sh_flag, unsigned char* smem) {
  ResHost* H = p.host;
  ResDevBlock* D = p.dev;
  const u32 t = threadIdx.x;
  for (;;) {
    if (t == 0) {
      u32 leave = 0;
      u64 w = 0;
      if (load_agent(&D->ctl.stop)) {
        leave = 1;
      } else {
        const u64 g = __hip_atomic_fetch_add(&D->ctl.gcursor, u64(1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const u64 tag = g & kResTagMask;
        u32 beat = load_agent(&D->ctl.beat);
        u64 beat_t = wall_clock64();
        // the shared stop and heartbeat words are read on every 8th poll only
        for (u32 n = 1;; ++n) {
          w = load_agent(&D->tiles[g & (kResTileRing - 1)]);
          if ((w >> 24) == tag) break;
          if ((n & 7) == 0) {
            if (load_agent(&D->ctl.stop)) {
              leave = 1;
              break;
            }
            const u32 b = load_agent(&D->ctl.beat);
            const u64 now = wall_clock64();
            if (b != beat) {
              beat = b;
              beat_t = now;
            } else if (now - beat_t > p.stall_ticks) {
              leave = 1;   // no dispatcher is running
              break;
            }
          }
          __builtin_amdgcn_s_sleep(32);
        }
      }
      sh_word = w;
      sh_flag = leave;
    }
    __syncthreads();
    if (sh_flag) break;
    const u64 w = sh_word;
    const u32 slot = (u32)(w >> 12) & 0xfffu, i = (u32)w & 0xfffu;
    // one invalidate for the workgroup (the L1 is the compute unit's, the L2
    // the XCD's): the descriptor, the request's inputs and its tables are
    // read fresh.  What tiles of this loop write (the outputs of a phase, read
    // by the next) moves by device-scope loads and stores (LoopIO) and needs
    // no cache operation.
    if (t == 0) fence_acquire_agent();
    __syncthreads();
    copy_entry(&E, &D->dent[slot]);
    __syncthreads();
    u32 phase = 0;
    while (phase + 1 < E.nphases && i >= E.prefix[phase + 1]) ++phase;
    if (phase > 0) {
      if (t == 0) {
        const u64 t0 = wall_clock64();
        u32 timed_out = 0;
        while (load_agent(&D->dphase[slot * kResLineWords]) < phase) {
          if (wall_clock64() - t0 > p.wait_ticks) {
            timed_out = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        sh_flag = timed_out;
      }
      __syncthreads();
    }
    const bool failed = phase > 0 && sh_flag;
    if (!failed) {
      const u32 tile = i - E.prefix[phase];
      if (E.kind == RES_NTT) {
        if (E.limbs == 2) run_item<4, kLogP4, false, LoopIO>(E.job, E.m4, phase, tile, smem);
        else run_item<2, kLogP2, false, LoopIO>(E.job, E.m2, phase, tile, smem);
      } else {
        if (E.limbs == 2) blas_tile<4>(E, E.m4, E.s4, tile);
        else blas_tile<2>(E, E.m2, E.s2, tile);
      }
    }
    // this tile's device-scope stores are visible to every XCD before its
    // count is: every wave waits until its own stores have completed
    wait_own_stores();
    __syncthreads();
    if (t == 0) {
      if (failed) {
        store_agent(&D->dfail[slot], 1u);
        store_agent(&D->ctl.error, 1u);
        wait_own_stores();
      }
      const u32 old = __hip_atomic_fetch_add(&D->dcount[slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old + 1 == E.total) {
        fence_acquire_agent();   // the failures other tiles recorded
        const u32 f = load_agent(&D->dfail[slot]);
        store_agent(&D->dcount[slot], 0u);
        store_agent(&D->dfail[slot], 0u);
        store_agent(&D->dphase[slot * kResLineWords], 0u);
        __hip_atomic_fetch_add(&D->ctl.completed, u64(1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // every tile's output is visible to the host and its copies first
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        __hip_atomic_store(&H->done[slot], (E.seq + 1) | ((u64)f << 63), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      } else if (phase + 1 < E.nphases && old + 1 == E.prefix[phase + 1]) {
        // The last tile of its phase: tiles of a later phase wait for this
        // one, so every tile counted so far is of this phase or an earlier
        // one, and each wrote its outputs back before it counted.  The
        // store follows the add that observed all of them.
        store_agent(&D->dphase[slot * kResLineWords], phase + 1);
      }
    }
    __syncthreads();   // E and the shared words are rewritten by the next tile
  }
  if (t == 0) __hip_atomic_fetch_add(&D->ctl.exited, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

__global__ __launch_bounds__(kExecThreads) __attribute__((amdgpu_waves_per_eu(2))) void resident_kernel(ResParams p) {
  extern __shared__ __align__(16) unsigned char mw_res_smem[];
  __shared__ ResEntry entry;
  __shared__ u64 sh_word;
  __shared__ u32 sh_flag;
  if (blockIdx.x == 0) dispatch(p, sh_word, sh_flag);
  else work(p, entry, sh_word, sh_flag, mw_res_smem);
}

hipError_t resident_launch(const ResParams& p, u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(resident_kernel, dim3(grid), dim3(kExecThreads), kResLds, s, p);
  return hipGetLastError();
}

}  // namespace mw
