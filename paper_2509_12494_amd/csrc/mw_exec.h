// Internal interface of the batched executor, shared by the C ABI
// (mw_exec.hip) and the serving runtime (mw_serve.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/mwntt.h"
#include "mw_ntt_tile.h"

struct ntt_plan_s;  // defined in mw_ntt.hip

namespace mw {

// Accessors into an ntt_plan_s (defined in mw_ntt.hip).
struct PlanView {
  uint32_t log2n, limbs, flags, variant;
  const uint64_t* q;
  const void* tw_fwd;
  const void* tw_inv;
};
template <int W>
struct ModConst {
  Modulus<W> M;
  Tw<W> ninv, last;
};
// Per-width constants of a plan: exactly one of c8 / c4 / c2 is filled (by
// limb count), the others are left as they are.
bool plan_view(const ntt_plan_s* P, PlanView& v, ModConst<8>& c8, ModConst<4>& c4, ModConst<2>& c2);

enum { JOB_FWD = 0, JOB_INV = 1, JOB_MUL = 2 };
constexpr int kExecThreads = 256;
constexpr int kLogP8 = 1;   // points per lane, four-word moduli
constexpr int kLogP4 = 2;   // two-word moduli
constexpr int kLogP2 = 3;   // one-word moduli

struct JobDesc {
  u64 in, in2, out, scratch;
  u64 tw_fwd, tw_inv;
  u32 op, limbs, log_n, log_n1;
  u32 perm_out, perm_in;
  u32 lines_col, lines_row;
  u32 tiles[3];
  u32 nphases;
};

// Host-side description of one run: descriptors, tile list per phase, LDS
// per phase, scratch per job (bytes; JobDesc::scratch is filled in by the
// owner of the scratch memory).
// Tiles of four-word jobs go to their own list and kernel (their residues
// take twice the registers, which would lower the occupancy of every tile if
// one kernel ran both).
struct ExecPlan {
  std::vector<JobDesc> jobs;
  std::vector<ModConst<8>> m8;
  std::vector<ModConst<4>> m4;
  std::vector<ModConst<2>> m2;
  std::vector<uint2> items;        // tiles of one- and two-word jobs
  std::vector<uint2> items8;       // tiles of four-word jobs
  std::vector<size_t> scratch_bytes;
  u32 phase_begin[4] = {0, 0, 0, 0};
  u32 phase_begin8[4] = {0, 0, 0, 0};
  // per phase, the limb counts (bit `limbs`) present in `items`: a phase with
  // one width runs that width's kernel, a phase with both the kernel for both
  u32 phase_widths[3] = {0, 0, 0};
  u32 nphases = 0;
  size_t phase_lds[3] = {0, 0, 0};
  size_t phase_lds8[3] = {0, 0, 0};
};

// Validates the jobs and fills `out` (no device work).  Status as mwntt.h.
int exec_build(const ntt_job* jobs, uint32_t count, ExecPlan& out);
// Raises the kernels' LDS limit when a run needs more than 64 KiB (once).
hipError_t exec_prepare(const ExecPlan& plan);

// Device copies of a run's descriptors (d_items8 / d_m8 may be null when the
// run has no four-word job).
struct ExecDevice {
  const JobDesc* jobs;
  const uint2* items;
  const uint2* items8;
  const ModConst<8>* m8;
  const ModConst<4>* m4;
  const ModConst<2>* m2;
};
// Launches the phases of a run whose descriptors are already on the device:
// per phase one launch over the one- and two-word tiles and one over the
// four-word tiles (each only when the phase has such tiles).
hipError_t exec_launch(const ExecDevice& d, const ExecPlan& plan, hipStream_t s);

struct ExecParams {
  const JobDesc* jobs;
  const uint2* items;      // this launch's tiles: {job | limbs << 16, phase << 16 | tile}
  const ModConst<8>* mods8;
  const ModConst<4>* mods4;
  const ModConst<2>* mods2;
  // A run of one job: its descriptor and constants travel in the kernel
  // arguments instead of device memory (no upload before the first launch),
  // and tile = workgroup index (column phases in XCD order).
  u32 one;                 // 1: the fields below are used, jobs / items / mods* are not
  u32 one_phase;
  u32 one_xcd;             // the phase's tiles are column tiles
  u32 one_pad;
  JobDesc one_job;
  ModConst<8> one_m8;      // the one filled for the job's width
  ModConst<4> one_m4;
  ModConst<2> one_m2;
};
static_assert(sizeof(ExecParams) <= 4096, "kernel arguments are limited to 4 KiB");

// Launches the phases of a run of exactly one job with its descriptor in the
// kernel arguments (no device copy of the descriptors is needed).
hipError_t exec_launch_one(const ExecPlan& plan, hipStream_t s);

// Validate mode: enqueues the canonicality check of every job's inputs on s
// (see mw_set_validate).  MW_OK or a negative status.
int exec_validate(const ExecPlan& plan, hipStream_t s);

}  // namespace mw
