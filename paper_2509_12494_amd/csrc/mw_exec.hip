// Batched executor: many NTT jobs -- forward, inverse, or a fused negacyclic
// product NTT(a), NTT(b) -> point-wise Barrett mulmod -> INTT (Background,
// polynomial multiplication using NTT) -- of different lengths and modulus
// widths, run as one kernel launch per phase.
//
// Every job is split into phases of tiles (two-pass transforms: column pass
// and row pass; a product has three phases: the forward column passes of a
// and b, a fused row phase, the inverse column pass).  Launch k runs every
// job's phase-k tiles, one workgroup per tile, whatever their length or
// width; stream order provides the dependencies between phases.  A run is two
// or three launches (twice that when four-word jobs are mixed in: they run in
// a kernel of their own) with no allocation and no memset, so it can be captured
// in a hipGraph and replayed.
//
// Dependencies are not resolved inside one launch on purpose: the L2 caches of
// the 8 XCDs are not coherent with each other during a kernel, so a tile that
// waits for tiles on other XCDs must write back and invalidate L2 around every
// hand-off, which costs more than the launch it would save.
//
// Tiles have 256 lanes and 4 points per lane for two-word moduli, 8 for
// one-word and 2 for four-word moduli (the shapes the autotuner found best for
// batches).  A launch whose tiles all have one width runs a kernel of that
// width only, in which tiles whose lines fill the 256 lanes (transforms of
// 2^(8 + log2 points per lane) points and more) with a line length of
// 2^5 .. 2^9 run the tile code of the single-purpose kernels, specialised per
// line length; the other tiles, and every tile of a launch that mixes one-
// and two-word moduli, run the run-time line engine of mw_ntt_rt.h (one
// kernel holding the specialised tiles of both widths needs more registers
// than either alone, and spills).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mw_common.h"
#include "mw_exec.h"
#include "mw_exec_tiles.h"
#include "mw_ntt_rt.h"
#include "mw_validate.h"

namespace mw {

// Tiles of one- and two-word jobs; item {job | limbs << 16, phase << 16 | tile}.
// The width comes with the item, so the job descriptor and the modulus
// constants (both indexed by the job) load in parallel instead of one after
// the other.  Run-time line engine only (launches that mix the two widths).
__global__ __launch_bounds__(kExecThreads) __attribute__((amdgpu_waves_per_eu(4))) void exec_kernel(ExecParams ep) {
  extern __shared__ __align__(16) unsigned char mw_exec_smem[];
  const uint2 it = ep.items[blockIdx.x];
  const u32 job = it.x & 0xffffu, limbs = it.x >> 16, phase = it.y >> 16, tile = it.y & 0xffffu;
  const JobDesc J = ep.jobs[job];
  if (limbs == 2) run_item<4, kLogP4, false>(J, ep.mods4[job], phase, tile, mw_exec_smem);
  else run_item<2, kLogP2, false>(J, ep.mods2[job], phase, tile, mw_exec_smem);
}

template <int W>
__device__ __forceinline__ const ModConst<W>* mods_of(const ExecParams& ep) {
  if constexpr (W == 8) return ep.mods8;
  else if constexpr (W == 4) return ep.mods4;
  else return ep.mods2;
}
template <int W>
__device__ __forceinline__ const ModConst<W>& one_mods_of(const ExecParams& ep) {
  if constexpr (W == 8) return ep.one_m8;
  else if constexpr (W == 4) return ep.one_m4;
  else return ep.one_m2;
}

// Tiles of one width (W 32-bit words per residue), with the specialised tile
// code; four-word jobs always run here (their own launch: see ExecPlan).
template <int W>
__global__ __launch_bounds__(kExecThreads) __attribute__((amdgpu_waves_per_eu(4))) void exec_kernel_w(ExecParams ep) {
  extern __shared__ __align__(16) unsigned char mw_exec_smem[];
  const uint2 it = ep.items[blockIdx.x];
  const u32 job = it.x & 0xffffu, phase = it.y >> 16, tile = it.y & 0xffffu;
  const JobDesc J = ep.jobs[job];
  constexpr int LOGP = W == 8 ? kLogP8 : (W == 4 ? kLogP4 : kLogP2);
  run_item<W, LOGP, true>(J, mods_of<W>(ep)[job], phase, tile, mw_exec_smem);
}

// The tiles of a run of one job, whose descriptor and constants are kernel
// arguments (a kernel of its own: reading them through a pointer that may
// also point to device memory would move the constants into vector
// registers).  tile = workgroup index, column phases in XCD order.  Its runs
// are small, so it may take the registers of 3 waves per SIMD (at 4 the
// constants held in scalar registers push the two-word tiles into a spill).
template <int W>
__global__ __launch_bounds__(kExecThreads) __attribute__((amdgpu_waves_per_eu(3))) void exec_kernel_one(ExecParams ep) {
  extern __shared__ __align__(16) unsigned char mw_exec_smem[];
  constexpr int LOGP = W == 8 ? kLogP8 : (W == 4 ? kLogP4 : kLogP2);
  const u32 tile = ep.one_xcd ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  run_item<W, LOGP, true>(ep.one_job, one_mods_of<W>(ep), ep.one_phase, tile, mw_exec_smem);
}

// host twin of xcd_tile: the tile that position b of a run of n tiles takes
static u32 xcd_order(u32 b, u32 n) {
  const u32 full = n - n % 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

static size_t npad_of(u32 logl, u32 logp) {
  const size_t L = (size_t)1 << logl;
  return (logl > logp ? L + (L >> logp) : L) + 1;
}

int exec_build(const ntt_job* jobs, uint32_t count, ExecPlan& out) {
  if (!jobs || count == 0 || count > 65535) return MW_EINVAL;
  out = ExecPlan();
  out.jobs.resize(count);
  out.m8.resize(count);
  out.m4.resize(count);
  out.m2.resize(count);
  out.scratch_bytes.resize(count);
  for (uint32_t i = 0; i < count; ++i) {
    const ntt_job& jb = jobs[i];
    if (!jb.plan || !jb.in || !jb.out || jb.op > NTT_JOB_POLYMUL) return MW_EINVAL;
    if (jb.op == NTT_JOB_POLYMUL && !jb.in2) return MW_EINVAL;
    PlanView v;
    ModConst<8>& c8 = out.m8[i];
    ModConst<4>& c4 = out.m4[i];
    ModConst<2>& c2 = out.m2[i];
    c8 = {};
    c4 = {};
    c2 = {};
    if (!plan_view(jb.plan, v, c8, c4, c2)) return MW_EINVAL;
    if (v.variant) return MW_EINVAL;    // arithmetic-variant plans run the plain entry points only
    if (v.log2n < 6) return MW_ESIZE;   // two-pass tiles need N1, N2 >= 8
    if (jb.op == NTT_JOB_POLYMUL && check_modulus(v.q, v.limbs) != MW_OK) return MW_EMODULUS;
    JobDesc& d = out.jobs[i];
    d = {};
    d.in = (u64)jb.in;
    d.in2 = (u64)jb.in2;
    d.out = (u64)jb.out;
    d.tw_fwd = (u64)v.tw_fwd;
    d.tw_inv = (u64)v.tw_inv;
    d.op = jb.op == NTT_JOB_FORWARD ? JOB_FWD : (jb.op == NTT_JOB_INVERSE ? JOB_INV : JOB_MUL);
    d.limbs = v.limbs;
    d.log_n = v.log2n;
    d.log_n1 = v.log2n / 2;
    d.perm_out = !(v.flags & NTT_BITREV_OUT);
    d.perm_in = !(v.flags & NTT_BITREV_IN);
    const u32 logp = v.limbs == 4 ? kLogP8 : (v.limbs == 2 ? kLogP4 : kLogP2);
    const u32 l1 = d.log_n1, l2 = v.log2n - d.log_n1;
    const u32 tpl_c = 1u << (l1 - logp), tpl_r = 1u << (l2 - logp);
    d.lines_col = std::min<u32>(kExecThreads / tpl_c, 1u << l2);
    d.lines_row = std::min<u32>(kExecThreads / tpl_r, 1u << l1);
    const u32 ncol = (1u << l2) / d.lines_col, nrow = (1u << l1) / d.lines_row;
    const size_t rsz = 8 * (size_t)v.limbs;
    const size_t lds_c = d.lines_col * npad_of(l1, logp) * rsz, lds_r = d.lines_row * npad_of(l2, logp) * rsz;
    size_t* pl = v.limbs == 4 ? out.phase_lds8 : out.phase_lds;
    if (d.op == JOB_FWD) {
      d.nphases = 2; d.tiles[0] = ncol; d.tiles[1] = nrow;
      pl[0] = std::max(pl[0], lds_c);
      pl[1] = std::max(pl[1], lds_r);
    } else if (d.op == JOB_INV) {
      d.nphases = 2; d.tiles[0] = nrow; d.tiles[1] = ncol;
      pl[0] = std::max(pl[0], lds_r);
      pl[1] = std::max(pl[1], lds_c);
    } else {
      d.nphases = 3; d.tiles[0] = 2 * ncol; d.tiles[1] = nrow; d.tiles[2] = ncol;
      pl[0] = std::max(pl[0], lds_c);
      pl[1] = std::max(pl[1], 2 * lds_r);   // rows of a and b
      pl[2] = std::max(pl[2], lds_c);
    }
    out.scratch_bytes[i] = (d.op == JOB_MUL ? 2 : 1) * (rsz << v.log2n);
  }
  for (int k = 0; k < 3; ++k)
    if (out.phase_lds[k] > 160 * 1024 || out.phase_lds8[k] > 160 * 1024) return MW_ESIZE;
  // tiles, phase-major: launch k covers [phase_begin[k], phase_begin[k+1]).
  // Workgroup b of a launch runs on XCD b mod 8 and each XCD has its own L2;
  // neighbouring column tiles read parts of the same cache lines, so a job's
  // run of column tiles is laid out such that consecutive tiles share an XCD
  // (the order xcd_tile gives).  Row tiles keep their order: the tiles that
  // write one output line are already a multiple of 8 apart.
  // Four-word jobs' tiles go to items8 in the same order.
  for (u32 ph = 0; ph < 3; ++ph) {
    out.phase_begin[ph] = (u32)out.items.size();
    out.phase_begin8[ph] = (u32)out.items8.size();
    for (uint32_t i = 0; i < count; ++i) {
      const JobDesc& d = out.jobs[i];
      if (ph >= d.nphases) continue;
      std::vector<uint2>& list = d.limbs == 4 ? out.items8 : out.items;
      const bool col = d.op == JOB_FWD ? ph == 0 : (d.op == JOB_INV ? ph == 1 : ph != 1);
      const u32 n = d.tiles[ph];
      for (u32 b = 0; b < n; ++b) {
        const u32 t = col ? xcd_order(b, n) : b;
        list.push_back(make_uint2(i | (d.limbs << 16), (ph << 16) | t));
      }
      if (n && d.limbs != 4) out.phase_widths[ph] |= 1u << d.limbs;
    }
    if (out.items.size() > out.phase_begin[ph] || out.items8.size() > out.phase_begin8[ph]) out.nphases = ph + 1;
  }
  out.phase_begin[3] = (u32)out.items.size();
  out.phase_begin8[3] = (u32)out.items8.size();
  return MW_OK;
}

template <typename K>
static hipError_t raise_lds(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

hipError_t exec_prepare(const ExecPlan& plan) {
  const size_t lds = std::max(plan.phase_lds[0], std::max(plan.phase_lds[1], plan.phase_lds[2]));
  const size_t lds8 = std::max(plan.phase_lds8[0], std::max(plan.phase_lds8[1], plan.phase_lds8[2]));
  // once per kernel: the first run that needs the larger limit raises it
  if (lds > 65536) {
    static const hipError_t e = [] {
      hipError_t r = raise_lds(exec_kernel, 65537);
      if (r == hipSuccess) r = raise_lds(exec_kernel_w<2>, 65537);
      if (r == hipSuccess) r = raise_lds(exec_kernel_w<4>, 65537);
      if (r == hipSuccess) r = raise_lds(exec_kernel_one<2>, 65537);
      if (r == hipSuccess) r = raise_lds(exec_kernel_one<4>, 65537);
      return r;
    }();
    if (e != hipSuccess) return e;
  }
  if (lds8 > 65536) {
    static const hipError_t e8 = [] {
      const hipError_t r = raise_lds(exec_kernel_w<8>, 65537);
      return r == hipSuccess ? raise_lds(exec_kernel_one<8>, 65537) : r;
    }();
    if (e8 != hipSuccess) return e8;
  }
  return hipSuccess;
}

hipError_t exec_launch_one(const ExecPlan& plan, hipStream_t s) {
  if (plan.jobs.size() != 1) return hipErrorInvalidValue;
  const JobDesc& d = plan.jobs[0];
  ExecParams ep = {};
  ep.one = 1;
  ep.one_job = d;
  ep.one_m8 = plan.m8[0];
  ep.one_m4 = plan.m4[0];
  ep.one_m2 = plan.m2[0];
  for (u32 k = 0; k < d.nphases; ++k) {
    ep.one_phase = k;
    // the same column-phase rule as the item lists' XCD order
    ep.one_xcd = d.op == JOB_FWD ? k == 0 : (d.op == JOB_INV ? k == 1 : k != 1);
    const dim3 grid(d.tiles[k]), block(kExecThreads);
    if (d.limbs == 4) hipLaunchKernelGGL(exec_kernel_one<8>, grid, block, plan.phase_lds8[k], s, ep);
    else if (d.limbs == 2) hipLaunchKernelGGL(exec_kernel_one<4>, grid, block, plan.phase_lds[k], s, ep);
    else hipLaunchKernelGGL(exec_kernel_one<2>, grid, block, plan.phase_lds[k], s, ep);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t exec_launch(const ExecDevice& d, const ExecPlan& plan, hipStream_t s) {
  ExecParams ep = {};
  ep.jobs = d.jobs;
  ep.mods8 = d.m8;
  ep.mods4 = d.m4;
  ep.mods2 = d.m2;
  for (u32 k = 0; k < plan.nphases; ++k) {
    const u32 n = plan.phase_begin[k + 1] - plan.phase_begin[k];
    if (n) {
      ep.items = d.items + plan.phase_begin[k];
      const size_t lds = plan.phase_lds[k];
      const u32 widths = plan.phase_widths[k];
      if (widths == (1u << 2)) hipLaunchKernelGGL(exec_kernel_w<4>, dim3(n), dim3(kExecThreads), lds, s, ep);
      else if (widths == (1u << 1)) hipLaunchKernelGGL(exec_kernel_w<2>, dim3(n), dim3(kExecThreads), lds, s, ep);
      else hipLaunchKernelGGL(exec_kernel, dim3(n), dim3(kExecThreads), lds, s, ep);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    const u32 n8 = plan.phase_begin8[k + 1] - plan.phase_begin8[k];
    if (n8) {
      ep.items = d.items8 + plan.phase_begin8[k];
      hipLaunchKernelGGL(exec_kernel_w<8>, dim3(n8), dim3(kExecThreads), plan.phase_lds8[k], s, ep);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace mw

using namespace mw;

namespace mw {
// Validate mode: enqueue the canonicality checks of every job's inputs.
int exec_validate(const ExecPlan& plan, hipStream_t s) {
  for (size_t i = 0; i < plan.jobs.size(); ++i) {
    const JobDesc& d = plan.jobs[i];
    const u32* qw = d.limbs == 4 ? plan.m8[i].M.q : (d.limbs == 2 ? plan.m4[i].M.q : plan.m2[i].M.q);
    uint64_t q[4] = {0, 0, 0, 0};
    for (u32 k = 0; k < 2 * d.limbs; ++k) q[k / 2] |= (uint64_t)qw[k] << (32 * (k % 2));
    const uint64_t n = (uint64_t)1 << d.log_n;
    int st = validate_input(reinterpret_cast<const void*>(d.in), n, q, d.limbs, s);
    if (st == MW_OK && d.op == JOB_MUL) st = validate_input(reinterpret_cast<const void*>(d.in2), n, q, d.limbs, s);
    if (st != MW_OK) return st;
  }
  return MW_OK;
}
}  // namespace mw

struct ntt_batch_s {
  int device = 0;
  ExecPlan plan;
  JobDesc* d_jobs = nullptr;
  uint2* d_items = nullptr;
  uint2* d_items8 = nullptr;
  ModConst<8>* d_m8 = nullptr;
  ModConst<4>* d_m4 = nullptr;
  ModConst<2>* d_m2 = nullptr;
  void* d_scratch = nullptr;
};

namespace {

void free_batch(ntt_batch_s* B) {
  if (!B) return;
  if (B->d_jobs) (void)hipFree(B->d_jobs);
  if (B->d_items) (void)hipFree(B->d_items);
  if (B->d_items8) (void)hipFree(B->d_items8);
  if (B->d_m8) (void)hipFree(B->d_m8);
  if (B->d_m4) (void)hipFree(B->d_m4);
  if (B->d_m2) (void)hipFree(B->d_m2);
  if (B->d_scratch) (void)hipFree(B->d_scratch);
  delete B;
}

template <typename T>
int upload(T** dst, const std::vector<T>& v) {
  if (v.empty()) return MW_OK;
  if (hipMalloc(dst, sizeof(T) * v.size()) != hipSuccess) return MW_ENOMEM;
  if (hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) return MW_EDEVICE;
  return MW_OK;
}

}  // namespace

extern "C" int ntt_batch_create(ntt_batch_t* out, const ntt_job* jobs, uint32_t count) {
  if (!out) return MW_EINVAL;
  *out = nullptr;
  ntt_batch_s* B = new (std::nothrow) ntt_batch_s();
  if (!B) return MW_ENOMEM;
  int st = exec_build(jobs, count, B->plan);
  if (st != MW_OK) {
    delete B;
    return st;
  }
  if (hipGetDevice(&B->device) != hipSuccess) {
    delete B;
    return MW_EDEVICE;
  }
  // one scratch allocation, 256-byte aligned slices
  size_t total = 0;
  std::vector<size_t> off(count);
  for (uint32_t i = 0; i < count; ++i) {
    off[i] = total;
    total += (B->plan.scratch_bytes[i] + 255) & ~(size_t)255;
  }
  if (hipMalloc(&B->d_scratch, total) != hipSuccess) st = MW_ENOMEM;
  if (st == MW_OK)
    for (uint32_t i = 0; i < count; ++i) B->plan.jobs[i].scratch = (u64)((char*)B->d_scratch + off[i]);
  if (st == MW_OK) st = upload(&B->d_jobs, B->plan.jobs);
  if (st == MW_OK) st = upload(&B->d_items, B->plan.items);
  if (st == MW_OK) st = upload(&B->d_items8, B->plan.items8);
  if (st == MW_OK) st = upload(&B->d_m8, B->plan.m8);
  if (st == MW_OK) st = upload(&B->d_m4, B->plan.m4);
  if (st == MW_OK) st = upload(&B->d_m2, B->plan.m2);
  if (st == MW_OK && exec_prepare(B->plan) != hipSuccess) st = MW_EDEVICE;
  if (st != MW_OK) {
    free_batch(B);
    return st;
  }
  *out = B;
  return MW_OK;
}

extern "C" int ntt_batch_run(ntt_batch_t batch, void* stream) {
  if (!batch) return MW_EINVAL;
  // (a batch's descriptors are already in device memory, so even a batch of
  // one job runs from them: measured faster than the kernel-argument form)
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (validate_on()) {
    int st = validate_take();
    if (st == MW_OK) st = exec_validate(batch->plan, s);
    if (st != MW_OK) return st;
  }
  const ExecDevice d{batch->d_jobs, batch->d_items, batch->d_items8, batch->d_m8, batch->d_m4, batch->d_m2};
  return exec_launch(d, batch->plan, s) == hipSuccess
             ? MW_OK
             : MW_EDEVICE;
}

extern "C" int ntt_batch_info(ntt_batch_t batch, uint32_t* tiles, uint32_t* launches) {
  if (!batch) return MW_EINVAL;
  if (tiles) *tiles = (uint32_t)(batch->plan.items.size() + batch->plan.items8.size());
  if (launches) {
    const ExecPlan& P = batch->plan;
    uint32_t n = 0;
    for (u32 k = 0; k < P.nphases; ++k)
      n += (P.phase_begin[k + 1] > P.phase_begin[k]) + (P.phase_begin8[k + 1] > P.phase_begin8[k]);
    *launches = n;
  }
  return MW_OK;
}

extern "C" int ntt_batch_check(ntt_batch_t batch) {
  if (!batch) return MW_EINVAL;
  return hipDeviceSynchronize() == hipSuccess ? MW_OK : MW_EDEVICE;
}

extern "C" int ntt_batch_destroy(ntt_batch_t batch) {
  if (!batch) return MW_EINVAL;
  (void)hipDeviceSynchronize();
  free_batch(batch);
  return MW_OK;
}
