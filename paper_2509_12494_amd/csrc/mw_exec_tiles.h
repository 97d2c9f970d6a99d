// Tile bodies of the batched executor: one column, row or fused row tile of
// a job (JobDesc), shared by the executor's launch-per-phase kernels and the
// serving runtime's resident request loop.  Every function here is run by
// all kExecThreads lanes of a workgroup and synchronizes them only with
// workgroup barriers.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mw_exec.h"
#include "mw_ntt_rt.h"

namespace mw {

// Line lengths 2^5 .. 2^9 get the compile-time tile code.
constexpr u32 kFixedLogLMin = 5, kFixedLogLMax = 9;

// One column or row tile.  With FIXED, a tile whose lines fill the workgroup
// (lines * 2^(logl - LOGP) == kExecThreads, no idle lanes) and whose line
// length has compile-time code runs the tile code of the single-purpose
// kernels (stage loops unrolled, indices constant); any other tile the
// run-time line engine.
template <int W, int LOGP, int DIR, int MODE, bool FIXED, class IO = CachedIO>
__device__ __forceinline__ void run_tile(const NttParams<W>& p, Res<W>* lds, u32 tile) {
  static_assert(!FIXED || std::is_same_v<IO, CachedIO>, "the compile-time tiles use cached accesses");
  if constexpr (FIXED) {
    const u32 logl = MODE == MODE_COL ? p.log_n1 : p.log_n - p.log_n1;
    if (logl >= kFixedLogLMin && logl <= kFixedLogLMax && (p.lines << (logl - LOGP)) == kExecThreads) {
      switch (logl) {
        case 5: if constexpr (shape_ok<W, MODE>(5, LOGP)) ntt_tile<W, 5, LOGP, DIR, MODE>(p, lds, tile); return;
        case 6: if constexpr (shape_ok<W, MODE>(6, LOGP)) ntt_tile<W, 6, LOGP, DIR, MODE>(p, lds, tile); return;
        case 7: if constexpr (shape_ok<W, MODE>(7, LOGP)) ntt_tile<W, 7, LOGP, DIR, MODE>(p, lds, tile); return;
        case 8: if constexpr (shape_ok<W, MODE>(8, LOGP)) ntt_tile<W, 8, LOGP, DIR, MODE>(p, lds, tile); return;
        default: if constexpr (shape_ok<W, MODE>(9, LOGP)) ntt_tile<W, 9, LOGP, DIR, MODE>(p, lds, tile); return;
      }
    }
  }
  rt_tile<W, LOGP, DIR, MODE, IO>(p, lds, tile);
}

// Fused row tile of a product with the line length fixed at compile time and
// lines * L/P == kExecThreads: the steps of rt_fused_row (the last forward
// stages of a and of b on `lines` consecutive rows, their point-wise Barrett
// product, the first inverse stages, written back over a's rows) with every
// lane busy and every shift and stage count constant.
template <int W, int LOGP, int LOGL>
__device__ __forceinline__ void fixed_fused_row(const NttParams<W>& pf, const NttParams<W>& pi, const Res<W>* src2,
                                                Res<W>* lds, u32 tile) {
  using S = LineShape<LOGL, LOGP>;
  constexpr u32 L = S::L;
  constexpr int P = S::P;
  constexpr u32 lines = kExecThreads / S::TPL;
  const u32 t = threadIdx.x;
  const u32 line_id = t / S::TPL, lane = t % S::TPL;
  const u32 row0 = tile * lines;
  Res<W>* la = lds;
  Res<W>* lb = lds + lines * S::NPAD;
  const auto off = [&](u32 e) { return ((u64)(row0 + e / L) << LOGL) + (e & (L - 1)); };
  const auto slot = [&](u32 e) { return (e / L) * S::NPAD + pad_idx<LOGL, LOGP>(e & (L - 1)); };
  {
    // all 2P loads of a and b in flight before the first LDS write
    Res<W> va[P], vb[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const u32 e = t + (u32)k * kExecThreads;
      va[k] = ResIO<W>::load(pf.src + off(e));
      vb[k] = ResIO<W>::load(src2 + off(e));
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const u32 e = t + (u32)k * kExecThreads;
      la[slot(e)] = va[k];
      lb[slot(e)] = vb[k];
    }
  }
  __syncthreads();
  const u32 base = (1u << pf.log_n1) + row0 + line_id;
  line_stages<W, LOGL, LOGP, DIR_FWD>(la + line_id * S::NPAD, lane, base, pf.tw, pf, false, true);
  line_stages<W, LOGL, LOGP, DIR_FWD>(lb + line_id * S::NPAD, lane, base, pf.tw, pf, false, true);
  const auto pointwise = [&](auto norm) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const u32 idx = slot(t + (u32)k * kExecThreads);
      la[idx] = barrett_mul_t<W, decltype(norm)::value>(la[idx], lb[idx], pf.M);
    }
  };
  if (pf.M.shift) pointwise(std::true_type{});
  else pointwise(std::false_type{});
  __syncthreads();
  line_stages<W, LOGL, LOGP, DIR_INV>(la + line_id * S::NPAD, lane, base, pi.tw, pi, false, false);
  const auto all = [](u32) { return true; };
  copy_staged<W, P>(
      t, kExecThreads, all, [&](u32 e) { return la[slot(e)]; },
      [&](u32 e, const Res<W>& v) { ResIO<W>::store(pf.dst + off(e), v); });
}

// The fused row tile of a product: with FIXED and a tile that fills the
// workgroup, the compile-time version -- for two-word moduli only: with the
// one- and four-word kernels' other tiles it exceeds their registers and
// spills.
template <int W, int LOGP, bool FIXED, class IO = CachedIO>
__device__ __forceinline__ void run_fused_row(const NttParams<W>& pf, const NttParams<W>& pi, const Res<W>* src2,
                                              Res<W>* lds, u32 tile) {
  static_assert(!FIXED || std::is_same_v<IO, CachedIO>, "the compile-time tiles use cached accesses");
  if constexpr (FIXED && W == 4) {
    const u32 logl = pf.log_n - pf.log_n1;
    if (logl >= kFixedLogLMin && logl <= kFixedLogLMax && (pf.lines << (logl - LOGP)) == kExecThreads) {
      switch (logl) {
        case 5: if constexpr (shape_ok<W, MODE_ROW>(5, LOGP)) fixed_fused_row<W, LOGP, 5>(pf, pi, src2, lds, tile); return;
        case 6: if constexpr (shape_ok<W, MODE_ROW>(6, LOGP)) fixed_fused_row<W, LOGP, 6>(pf, pi, src2, lds, tile); return;
        case 7: if constexpr (shape_ok<W, MODE_ROW>(7, LOGP)) fixed_fused_row<W, LOGP, 7>(pf, pi, src2, lds, tile); return;
        case 8: if constexpr (shape_ok<W, MODE_ROW>(8, LOGP)) fixed_fused_row<W, LOGP, 8>(pf, pi, src2, lds, tile); return;
        default: if constexpr (shape_ok<W, MODE_ROW>(9, LOGP)) fixed_fused_row<W, LOGP, 9>(pf, pi, src2, lds, tile); return;
      }
    }
  }
  rt_fused_row<W, LOGP, IO>(pf, pi, src2, lds, tile);
}

template <int W, int LOGP, bool FIXED, class IO = CachedIO>
__device__ __forceinline__ void run_item(const JobDesc& J, const ModConst<W>& mc, u32 phase, u32 tile,
                                         unsigned char* smem) {
  NttParams<W> p;
  p.M = mc.M;
  p.ninv = mc.ninv;
  p.ninv_w1 = mc.last;
  p.log_n = J.log_n;
  p.log_n1 = J.log_n1;
  p.batch = 1;
  p.permute = 0;
  Res<W>* lds = reinterpret_cast<Res<W>*>(smem);
  const u64 N = (u64)1 << J.log_n;
  const Res<W>* in = reinterpret_cast<const Res<W>*>(J.in);
  const Res<W>* in2 = reinterpret_cast<const Res<W>*>(J.in2);
  Res<W>* out = reinterpret_cast<Res<W>*>(J.out);
  Res<W>* scr = reinterpret_cast<Res<W>*>(J.scratch);
  const Tw<W>* twf = reinterpret_cast<const Tw<W>*>(J.tw_fwd);
  const Tw<W>* twi = reinterpret_cast<const Tw<W>*>(J.tw_inv);
  if (J.op == JOB_FWD) {
    p.tw = twf;
    if (phase == 0) {
      p.src = in; p.dst = scr; p.lines = J.lines_col;
      run_tile<W, LOGP, DIR_FWD, MODE_COL, FIXED, IO>(p, lds, tile);
    } else {
      p.src = scr; p.dst = out; p.lines = J.lines_row; p.permute = J.perm_out;
      run_tile<W, LOGP, DIR_FWD, MODE_ROW, FIXED, IO>(p, lds, tile);
    }
  } else if (J.op == JOB_INV) {
    p.tw = twi;
    if (phase == 0) {
      p.src = in; p.dst = scr; p.lines = J.lines_row; p.permute = J.perm_in;
      run_tile<W, LOGP, DIR_INV, MODE_ROW, FIXED, IO>(p, lds, tile);
    } else {
      p.src = scr; p.dst = out; p.lines = J.lines_col;
      run_tile<W, LOGP, DIR_INV, MODE_COL, FIXED, IO>(p, lds, tile);
    }
  } else {
    const u32 ncol = J.tiles[2];
    if (phase == 0) {
      p.tw = twf; p.lines = J.lines_col;
      const bool second = tile >= ncol;
      p.src = second ? in2 : in;
      p.dst = second ? scr + N : scr;
      run_tile<W, LOGP, DIR_FWD, MODE_COL, FIXED, IO>(p, lds, second ? tile - ncol : tile);
    } else if (phase == 1) {
      NttParams<W> pi = p;
      p.tw = twf; p.lines = J.lines_row; p.src = scr; p.dst = scr;
      pi.tw = twi; pi.lines = J.lines_row;
      run_fused_row<W, LOGP, FIXED, IO>(p, pi, scr + N, lds, tile);
    } else {
      p.tw = twi; p.lines = J.lines_col; p.src = scr; p.dst = out;
      run_tile<W, LOGP, DIR_INV, MODE_COL, FIXED, IO>(p, lds, tile);
    }
  }
}

}  // namespace mw
