// NTT line engine with the line length chosen at run time.
//
// Same algorithm, butterflies and LDS layout as the compile-time tiles of
// mw_ntt_tile.h (see the notes there), but log2 of the line length is a
// run-time value and only the points per lane (2^LOGP) is a template
// parameter: a round of LOGP stages is one compile-time code path whose
// shifts and twiddle indices use the run-time stage offset, and the first
// round, holding the remaining log2(L) mod LOGP stages, has its own path per
// remainder.  One kernel can then run lines of every length, which the
// persistent executor needs (jobs of different N in one launch).
//
// Workgroups may be wider than a tile (lines * L/P lanes): lanes beyond it are
// inactive but still reach every barrier.
#pragma once
#include "mw_ntt_tile.h"

namespace mw {

template <int LOGP>
__device__ __forceinline__ u32 rt_pad(u32 j, u32 logl) {
  return logl > (u32)LOGP ? j + (j >> LOGP) : j;
}

__device__ __forceinline__ u32 rt_npad(u32 logl, u32 logp) {
  const u32 L = 1u << logl;
  return (logl > logp ? L + (L >> logp) : L) + 1;
}

// One round of NP stages (NP <= LOGP) starting at stage s0 of the line.
// LAST_INV: the round may hold the final inverse stage (stage 0, N^-1 folded
// in); CANON: make the outputs canonical.  Both are known where a round is
// called, so rounds without them carry no code for them.
template <int W, int LOGP, int NP, int DIR, bool LAST_INV, bool CANON, class IO = CachedIO>
__device__ __forceinline__ void rt_round(Res<W>* line, bool active, u32 logl, u32 s0, u32 tid, u32 base,
                                         const Tw<W>* __restrict__ tw, const NttParams<W>& p) {
  constexpr int P = 1 << LOGP;
  if (active) {
    const u32 L0 = logl - s0 - LOGP;
    const u32 base_j = ((tid >> L0) << (L0 + LOGP)) | (tid & ((1u << L0) - 1u));
    Res<W> x[P];
#pragma unroll
    for (int u = 0; u < P; ++u) x[u] = line[rt_pad<LOGP>(base_j | ((u32)u << L0), logl)];
#pragma unroll
    for (int st0 = 0; st0 < NP; ++st0) {
      const int st = (DIR == DIR_FWD) ? st0 : (NP - 1 - st0);
      const u32 s = s0 + st;
      const int ib = LOGP - 1 - st;
      const int ngroups = 1 << st;
#pragma unroll
      for (int gi = 0; gi < ngroups; ++gi) {
        const u32 j0 = base_j | ((u32)(gi << (ib + 1)) << L0);
        const u32 g = j0 >> (logl - s);
        if (DIR == DIR_INV && LAST_INV && s == 0) {
#pragma unroll
          for (int lo = 0; lo < (1 << ib); ++lo) {
            const int u = (gi << (ib + 1)) | lo;
            gs_bfly_last(x[u], x[u | (1 << ib)], p.ninv, p.ninv_w1, p.M);
          }
        } else {
          const Tw<W> t = IO::tw(tw, (base << s) + g);
#pragma unroll
          for (int lo = 0; lo < (1 << ib); ++lo) {
            const int u = (gi << (ib + 1)) | lo;
            if (DIR == DIR_FWD) ct_bfly(x[u], x[u | (1 << ib)], t, p.M);
            else gs_bfly(x[u], x[u | (1 << ib)], t, p.M);
          }
        }
      }
    }
    if constexpr (CANON) {
#pragma unroll
      for (int u = 0; u < P; ++u) x[u] = canon16(x[u], p.M);
    }
#pragma unroll
    for (int u = 0; u < P; ++u) line[rt_pad<LOGP>(base_j | ((u32)u << L0), logl)] = x[u];
  }
  __syncthreads();
}

template <int W, int LOGP, int DIR, bool LAST_INV, bool CANON, class IO = CachedIO>
__device__ __forceinline__ void rt_first_round(u32 p0, Res<W>* line, bool active, u32 logl, u32 tid, u32 base,
                                               const Tw<W>* __restrict__ tw, const NttParams<W>& p) {
  // p0 in [1, LOGP]: stages 0 .. p0-1 of the line
  if constexpr (LOGP >= 1) {
    if (p0 == 1) { rt_round<W, LOGP, 1, DIR, LAST_INV, CANON, IO>(line, active, logl, 0, tid, base, tw, p); return; }
  }
  if constexpr (LOGP >= 2) {
    if (p0 == 2) { rt_round<W, LOGP, 2, DIR, LAST_INV, CANON, IO>(line, active, logl, 0, tid, base, tw, p); return; }
  }
  if constexpr (LOGP >= 3) {
    if (p0 == 3) { rt_round<W, LOGP, 3, DIR, LAST_INV, CANON, IO>(line, active, logl, 0, tid, base, tw, p); return; }
  }
  if constexpr (LOGP >= 4) {
    rt_round<W, LOGP, 4, DIR, LAST_INV, CANON, IO>(line, active, logl, 0, tid, base, tw, p);
  }
}

// All stages of a line of 2^logl points (logl >= LOGP) held in LDS.
// LAST_INV: the line holds the final inverse stage; FINAL_FWD: canonicalize
// after the last forward stage.
template <int W, int LOGP, int DIR, bool LAST_INV, bool FINAL_FWD, class IO = CachedIO>
__device__ __forceinline__ void rt_line_stages(Res<W>* line, bool active, u32 logl, u32 tid, u32 base,
                                               const Tw<W>* __restrict__ tw, const NttParams<W>& p) {
  const u32 R = (logl + LOGP - 1) / LOGP;
  const u32 p0 = logl - LOGP * (R - 1);
  if (DIR == DIR_FWD) {
    if (R == 1) {
      rt_first_round<W, LOGP, DIR, false, FINAL_FWD, IO>(p0, line, active, logl, tid, base, tw, p);
      return;
    }
    rt_first_round<W, LOGP, DIR, false, false, IO>(p0, line, active, logl, tid, base, tw, p);
    for (u32 r = 1; r + 1 < R; ++r)
      rt_round<W, LOGP, LOGP, DIR, false, false, IO>(line, active, logl, p0 + (r - 1) * LOGP, tid, base, tw, p);
    rt_round<W, LOGP, LOGP, DIR, false, FINAL_FWD, IO>(line, active, logl, p0 + (R - 2) * LOGP, tid, base, tw, p);
  } else {
    // only the first round holds stage 0
    for (u32 r = R - 1; r >= 1; --r)
      rt_round<W, LOGP, LOGP, DIR, false, false, IO>(line, active, logl, p0 + (r - 1) * LOGP, tid, base, tw, p);
    rt_first_round<W, LOGP, DIR, LAST_INV, false, IO>(p0, line, active, logl, tid, base, tw, p);
  }
}

// One column or row tile of a single transform (batch index 0 of p.src /
// p.dst), with run-time line length.  `tile` indexes the tiles of the pass.
template <int W, int LOGP, int DIR, int MODE, class IO = CachedIO>
__device__ __forceinline__ void rt_tile(const NttParams<W>& p, Res<W>* lds, u32 tile) {
  static_assert(MODE == MODE_COL || MODE == MODE_ROW, "two-pass tiles only");
  const u32 log_n = p.log_n, log_n1 = p.log_n1, log_n2 = log_n - log_n1;
  const u32 logl = MODE == MODE_COL ? log_n1 : log_n2;
  const u32 L = 1u << logl;
  const u32 npad = rt_npad(logl, LOGP);
  const u32 lines = p.lines;
  const u32 log_lines = __builtin_ctz(lines);
  const u32 tpl = L >> LOGP;
  const u32 T = lines * tpl;
  const u32 t = threadIdx.x;
  const bool active = t < T;
  const u32 line_id = active ? t / tpl : 0;
  const u32 lane = t % tpl;
  const u32 nelem = lines << logl;
  const u32 nthreads = blockDim.x;

  u32 c0 = 0, b_lo = 0;
  if (MODE == MODE_COL) c0 = tile * lines;
  else b_lo = tile;

  // ---- device memory -> LDS ----
  constexpr int P = 1 << LOGP;
  const auto in_tile = [&](u32 e) { return e < nelem; };
  if (MODE == MODE_COL) {
    const u64 N2 = (u64)1 << log_n2;
    copy_staged<W, P>(
        t, nthreads, in_tile,
        [&](u32 e) { return IO::load(p.src + (e >> log_lines) * N2 + c0 + (e & (lines - 1))); },
        [&](u32 e, const Res<W>& v) { lds[(e & (lines - 1)) * npad + rt_pad<LOGP>(e >> log_lines, logl)] = v; });
  } else {
    const u32 n1_over_g = (1u << log_n1) >> log_lines;
    if (DIR == DIR_INV && p.permute) {
      const u32 col = brev(b_lo, log_n1 - log_lines) << log_lines;
      copy_staged<W, P>(
          t, nthreads, in_tile,
          [&](u32 e) { return IO::load(p.src + ((u64)(e >> log_lines) << log_n1) + col + (e & (lines - 1))); },
          [&](u32 e, const Res<W>& v) {
            lds[brev(e & (lines - 1), log_lines) * npad + rt_pad<LOGP>(brev(e >> log_lines, logl), logl)] = v;
          });
    } else {
      copy_staged<W, P>(
          t, nthreads, in_tile,
          [&](u32 e) {
            const u32 b = (e >> logl) * n1_over_g + b_lo;
            return IO::load(p.src + ((u64)b << logl) + (e & (L - 1)));
          },
          [&](u32 e, const Res<W>& v) { lds[(e >> logl) * npad + rt_pad<LOGP>(e & (L - 1), logl)] = v; });
    }
  }
  __syncthreads();

  u32 base = 1;
  if (MODE == MODE_ROW) base = (1u << log_n1) + line_id * ((1u << log_n1) >> log_lines) + b_lo;
  rt_line_stages<W, LOGP, DIR, DIR == DIR_INV && MODE != MODE_ROW, DIR == DIR_FWD && MODE != MODE_COL, IO>(
      lds + line_id * npad, active, logl, lane, base, p.tw, p);

  // ---- LDS -> device memory ----
  if (MODE == MODE_COL) {
    const u64 N2 = (u64)1 << log_n2;
    copy_staged<W, P>(
        t, nthreads, in_tile,
        [&](u32 e) { return lds[(e & (lines - 1)) * npad + rt_pad<LOGP>(e >> log_lines, logl)]; },
        [&](u32 e, const Res<W>& v) { IO::store(p.dst + (e >> log_lines) * N2 + c0 + (e & (lines - 1)), v); });
  } else {
    const u32 n1_over_g = (1u << log_n1) >> log_lines;
    if (DIR == DIR_FWD && p.permute) {
      const u32 col = brev(b_lo, log_n1 - log_lines) << log_lines;
      copy_staged<W, P>(
          t, nthreads, in_tile,
          [&](u32 e) {
            return lds[brev(e & (lines - 1), log_lines) * npad + rt_pad<LOGP>(brev(e >> log_lines, logl), logl)];
          },
          [&](u32 e, const Res<W>& v) {
            IO::store(p.dst + ((u64)(e >> log_lines) << log_n1) + col + (e & (lines - 1)), v);
          });
    } else {
      copy_staged<W, P>(
          t, nthreads, in_tile, [&](u32 e) { return lds[(e >> logl) * npad + rt_pad<LOGP>(e & (L - 1), logl)]; },
          [&](u32 e, const Res<W>& v) {
            const u32 b = (e >> logl) * n1_over_g + b_lo;
            IO::store(p.dst + ((u64)b << logl) + (e & (L - 1)), v);
          });
    }
  }
}

// Fused row tile of a negacyclic product: the last log N2 forward stages of
// a (p.src) and of b (src2) on the same `lines` consecutive rows, their
// point-wise Barrett product, then the first log N2 inverse stages, written
// back over a's rows.  Everything stays in bit-reversed order, which is the
// order the inverse's row pass takes, so no permutation is needed.  `lds`
// holds 2 * lines * npad residues.  `pi` carries the inverse table and N^-1.
template <int W, int LOGP, class IO = CachedIO>
__device__ __forceinline__ void rt_fused_row(const NttParams<W>& pf, const NttParams<W>& pi, const Res<W>* src2,
                                             Res<W>* lds, u32 tile) {
  const u32 log_n = pf.log_n, log_n1 = pf.log_n1, log_n2 = log_n - log_n1;
  const u32 logl = log_n2;
  const u32 L = 1u << logl;
  const u32 npad = rt_npad(logl, LOGP);
  const u32 lines = pf.lines;
  const u32 tpl = L >> LOGP;
  const u32 T = lines * tpl;
  const u32 t = threadIdx.x;
  const bool active = t < T;
  const u32 line_id = active ? t / tpl : 0;
  const u32 lane = t % tpl;
  const u32 nelem = lines << logl;
  const u32 nthreads = blockDim.x;
  const u32 row0 = tile * lines;
  Res<W>* la = lds;
  Res<W>* lb = lds + lines * npad;

  constexpr int P = 1 << LOGP;
  const auto in_tile = [&](u32 e) { return e < nelem; };
  const auto off = [&](u32 e) { return ((u64)(row0 + (e >> logl)) << logl) + (e & (L - 1)); };
  const auto slot = [&](u32 e) { return (e >> logl) * npad + rt_pad<LOGP>(e & (L - 1), logl); };
  {
    // all 2P loads of a and b in flight before the first LDS write
    Res<W> va[P], vb[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const u32 e = t + (u32)k * nthreads;
      if (in_tile(e)) {
        va[k] = IO::load(pf.src + off(e));
        vb[k] = IO::load(src2 + off(e));
      }
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const u32 e = t + (u32)k * nthreads;
      if (in_tile(e)) {
        la[slot(e)] = va[k];
        lb[slot(e)] = vb[k];
      }
    }
  }
  __syncthreads();
  const u32 base = (1u << log_n1) + row0 + line_id;
  rt_line_stages<W, LOGP, DIR_FWD, false, true, IO>(la + line_id * npad, active, logl, lane, base, pf.tw, pf);
  rt_line_stages<W, LOGP, DIR_FWD, false, true, IO>(lb + line_id * npad, active, logl, lane, base, pf.tw, pf);
  // point-wise Barrett products; the scaled or plain form is chosen once for
  // the loop (a uniform branch on the job's modulus)
  const auto pointwise = [&](auto norm) {
    for (u32 e = t; e < nelem; e += nthreads) {
      const u32 j = e >> logl, l = e & (L - 1);
      const u32 idx = j * npad + rt_pad<LOGP>(l, logl);
      la[idx] = barrett_mul_t<W, decltype(norm)::value>(la[idx], lb[idx], pf.M);
    }
  };
  if (pf.M.shift) pointwise(std::true_type{});
  else pointwise(std::false_type{});
  __syncthreads();
  rt_line_stages<W, LOGP, DIR_INV, false, false, IO>(la + line_id * npad, active, logl, lane, base, pi.tw, pi);
  copy_staged<W, P>(
      t, nthreads, in_tile, [&](u32 e) { return la[slot(e)]; },
      [&](u32 e, const Res<W>& v) { IO::store(pf.dst + off(e), v); });
}

}  // namespace mw
