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
  uint32_t log2n, limbs, flags;
  const uint64_t* q;
  const void* tw_fwd;
  const void* tw_inv;
};
bool plan_view(const ntt_plan_s* P, PlanView& v, Modulus<4>& m4, Tw<4>& n4, Tw<4>& l4, Modulus<2>& m2, Tw<2>& n2,
               Tw<2>& l2);

enum { JOB_FWD = 0, JOB_INV = 1, JOB_MUL = 2 };
constexpr int kExecThreads = 256;
constexpr int kLogP4 = 2;   // points per lane, two-word moduli
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

template <int W>
struct ModConst {
  Modulus<W> M;
  Tw<W> ninv, last;
};

// Host-side description of one run: descriptors, tile list per phase, LDS
// per phase, scratch per job (bytes; JobDesc::scratch is filled in by the
// owner of the scratch memory).
struct ExecPlan {
  std::vector<JobDesc> jobs;
  std::vector<ModConst<4>> m4;
  std::vector<ModConst<2>> m2;
  std::vector<uint2> items;
  std::vector<size_t> scratch_bytes;
  u32 phase_begin[4] = {0, 0, 0, 0};
  u32 nphases = 0;
  size_t phase_lds[3] = {0, 0, 0};
};

// Validates the jobs and fills `out` (no device work).  Status as mwntt.h.
int exec_build(const ntt_job* jobs, uint32_t count, ExecPlan& out);
// Raises the kernel's LDS limit when a run needs more than 64 KiB (once).
hipError_t exec_prepare(size_t max_lds);
// Launches the phases of a run whose descriptors are already on the device.
hipError_t exec_launch(const JobDesc* d_jobs, const uint2* d_items, const ModConst<4>* d_m4,
                       const ModConst<2>* d_m2, const ExecPlan& plan, hipStream_t s);

struct ExecParams {
  const JobDesc* jobs;
  const uint2* items;      // this launch's tiles: {job, phase << 16 | tile}
  const ModConst<4>* mods4;
  const ModConst<2>* mods2;
};

}  // namespace mw
