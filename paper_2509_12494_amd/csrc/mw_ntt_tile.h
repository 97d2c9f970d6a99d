// Negacyclic NTT / INTT tiles over Z_q[X]/(X^N + 1) for gfx950.
//
// What is computed (Background, polynomial multiplication using NTT, Eq. ntt):
//   forward  A_k = sum_j a_j psi^(j(2k+1))             (Eq. ntt on a_j psi^j,
//   inverse  a_j = N^-1 psi^-j sum_k A_k psi^(-2jk)      omega_N = psi^2)
// An N-point transform is log N stages of N/2 butterflies, each one modular
// multiplication, one addition and one subtraction (SIMD-vectorized kernels,
// from arithmetic to cryptographic kernels).
//
// Algorithm.  The forward transform is the merged-psi Cooley-Tukey form:
// stage s (m = 2^s groups, half-width t = N/2m) pairs j and j+t and
// multiplies by tw[m + floor(j/2t)], tw[i] = psi^bitrev(i), leaving the output
// in bit-reversed order.  The inverse is the Gentleman-Sande form with
// tw'[i] = psi^-bitrev(i), processing the stages in reverse and taking
// bit-reversed input; N^-1 is folded into its last stage.  Butterflies are
// lazy (Harvey): forward values stay in [0, 16q), inverse values in [0, 8q),
// with one conditional subtraction per butterfly; results are made canonical
// once at the end.
//
// Data movement (the paper permutes between stages with AVX-512 unpack /
// permute instructions; here stages exchange data through LDS):
//   * a "line" is an n = 2^LOGL point sub-transform held by n/P lanes, each lane
//     owning P = 2^LOGP points; LOGP stages run in registers per round, and
//     lanes exchange points through LDS between rounds;
//   * small N: one line per transform, the whole transform in one workgroup
//     ("full" tiles);
//   * larger N: N = N1 * N2 and two passes over device memory.  The first
//     log N1 Cooley-Tukey stages only pair elements in the same residue class
//     mod N2 (columns of stride N2) and use the table entries below N1, so a
//     column is an N1-point line with twiddle base 1.  The remaining log N2
//     stages act within contiguous rows of N2 elements; row b is an N2-point
//     line whose local stage m' uses tw[m' * (N1 + b) + g].  No transpose and
//     no extra twiddle pass are needed.  The inverse runs the rows first, then
//     the columns.
//   * natural-order output of the forward transform: row b, local index l
//     holds A at k = bitrev(l)*N1 + bitrev(b).  A row tile takes G rows
//     b = j*(N1/G) + b_lo, whose outputs land in runs of G consecutive
//     residues, so the permuted store (and the inverse's permuted load) is
//     coalesced in G-residue segments.
// The number of lines per tile (columns, rows or whole transforms) is a
// launch-time choice; the points per lane P is a template parameter.
#pragma once
#include <hip/hip_runtime.h>

#include "mw_arith.h"
#include "mw_butterfly.h"

namespace mw {

template <int W>
__device__ __forceinline__ Tw<W> load_tw(const Tw<W>* t, u32 idx) {
  Tw<W> r;
  if constexpr (W == 8) {
    const uint4* p = reinterpret_cast<const uint4*>(t + idx);
    const uint4 a0 = p[0], a1 = p[1], b0 = p[2], b1 = p[3];
    r.w[0] = a0.x; r.w[1] = a0.y; r.w[2] = a0.z; r.w[3] = a0.w;
    r.w[4] = a1.x; r.w[5] = a1.y; r.w[6] = a1.z; r.w[7] = a1.w;
    r.ws[0] = b0.x; r.ws[1] = b0.y; r.ws[2] = b0.z; r.ws[3] = b0.w;
    r.ws[4] = b1.x; r.ws[5] = b1.y; r.ws[6] = b1.z; r.ws[7] = b1.w;
  } else if constexpr (W == 4) {
    const uint4* p = reinterpret_cast<const uint4*>(t + idx);
    uint4 a = p[0], b = p[1];
    r.w[0] = a.x; r.w[1] = a.y; r.w[2] = a.z; r.w[3] = a.w;
    r.ws[0] = b.x; r.ws[1] = b.y; r.ws[2] = b.z; r.ws[3] = b.w;
  } else {
    uint4 a = *reinterpret_cast<const uint4*>(t + idx);
    r.w[0] = a.x; r.w[1] = a.y;
    r.ws[0] = a.z; r.ws[1] = a.w;
  }
  return r;
}

// Device-memory access of the run-time tile bodies (mw_ntt_rt.h), as a
// template policy: load and store move the residues a tile transforms, tw
// reads its twiddle table.
//
// CachedIO: ordinary loads and stores through the compute unit's L1 and the
// XCD's L2, for kernels whose workgroups exchange data only across launches.
//
// LoopIO, for the persistent request loop, where a tile reads what tiles on
// other XCDs wrote in the same launch: residues move as relaxed device-scope
// atomics on 64-bit words.  Such a load does not return a line the L1 or the
// XCD's L2 holds from before another XCD's write, and such a store is written
// through to memory, so that once the writing wave has waited for its stores
// they are visible to every XCD: neither side needs an L2 invalidate or
// write-back for them.  Twiddle tables, which no tile writes, are read
// through the caches.
struct CachedIO {
  template <int W>
  __device__ static __forceinline__ Res<W> load(const Res<W>* p) { return ResIO<W>::load(p); }
  template <int W>
  __device__ static __forceinline__ void store(Res<W>* p, const Res<W>& v) { ResIO<W>::store(p, v); }
  template <int W>
  __device__ static __forceinline__ Tw<W> tw(const Tw<W>* t, u32 idx) { return load_tw(t, idx); }
};

struct LoopIO {
  template <int W>
  __device__ static __forceinline__ Res<W> load(const Res<W>* p) {
    static_assert(W % 2 == 0, "whole 64-bit words");
    u64* s = reinterpret_cast<u64*>(const_cast<Res<W>*>(p));
    Res<W> r;
#pragma unroll
    for (int k = 0; k < W / 2; ++k) {
      const u64 x = __hip_atomic_load(s + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      r.v[2 * k] = (u32)x;
      r.v[2 * k + 1] = (u32)(x >> 32);
    }
    return r;
  }
  template <int W>
  __device__ static __forceinline__ void store(Res<W>* p, const Res<W>& v) {
    static_assert(W % 2 == 0, "whole 64-bit words");
    u64* d = reinterpret_cast<u64*>(p);
#pragma unroll
    for (int k = 0; k < W / 2; ++k)
      __hip_atomic_store(d + k, (u64)v.v[2 * k] | ((u64)v.v[2 * k + 1] << 32), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  template <int W>
  __device__ static __forceinline__ Tw<W> tw(const Tw<W>* t, u32 idx) { return load_tw(t, idx); }
};

enum { DIR_FWD = 0, DIR_INV = 1 };
enum { MODE_FULL = 0, MODE_COL = 1, MODE_ROW = 2 };

template <int W>
struct NttParams {
  const Res<W>* src;     // input of this pass
  Res<W>* dst;           // output of this pass
  const Tw<W>* tw;       // this direction's table, N entries
  Modulus<W> M;
  Tw<W> ninv;            // N^-1 and its Shoup companion (inverse only)
  Tw<W> ninv_w1;         // tw'[1] * N^-1 (inverse only)
  u32 log_n;             // transform size
  u32 log_n1;            // rows of the two-pass split (N1 = 2^log_n1)
  u32 batch;             // transforms in this launch
  u32 permute;           // 1: natural order at the device-memory side of this pass
  u32 lines;             // lines per tile (a power of two)
  u32 pad_[3];
};

__device__ __forceinline__ u32 brev(u32 x, u32 bits) {
  return bits ? (__builtin_bitreverse32(x) >> (32 - bits)) : 0u;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b mod 8), and each XCD has its own L2.  Neighbouring column tiles of a
// few columns each read parts of the same 128-byte lines, so map workgroups to
// tiles such that consecutive tiles run on the same XCD: within the largest
// multiple of 8 workgroups, workgroup b takes tile (b mod 8) * (n / 8) + b / 8;
// the remainder keeps its index.  A bijection on [0, n).  (Measured with the
// FETCH_SIZE counter: it removes the 2x / 4x over-fetch of 4- / 2-column
// tiles.)
constexpr u32 kXcds = 8;
__device__ __forceinline__ u32 xcd_tile(u32 b, u32 n) {
  const u32 full = n - n % kXcds;
  if (b >= full) return b;
  return (b % kXcds) * (full / kXcds) + b / kXcds;
}

// Tile <-> LDS copies.  Thread t moves elements e = t + k*nthreads for
// k < P (a tile of `lines` lines of L points moved by lines*L/P threads is
// exactly P elements per thread; the run-time engine may have fewer).  All P
// reads are issued before the first write, so the P device-memory loads (or
// LDS reads) of a thread are in flight together instead of one at a time.
// rd(e) reads element e, wr(e, v) writes it; ok(e) guards both.
template <int W, int P, class Ok, class Rd, class Wr>
__device__ __forceinline__ void copy_staged(u32 t, u32 nthreads, Ok ok, Rd rd, Wr wr) {
  Res<W> v[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const u32 e = t + (u32)k * nthreads;
    if (ok(e)) v[k] = rd(e);
  }
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const u32 e = t + (u32)k * nthreads;
    if (ok(e)) wr(e, v[k]);
  }
}

template <int LOGL, int LOGP>
struct LineShape {
  static constexpr int L = 1 << LOGL;
  static constexpr int P = 1 << LOGP;
  static constexpr int TPL = L / P;                      // lanes per line
  // line stride in LDS: one padding slot per P points, plus one so that the
  // same point of consecutive lines falls in different banks
  static constexpr int NPAD = ((LOGL > LOGP) ? L + L / P : L) + 1;
  static constexpr int R = (LOGL + LOGP - 1) / LOGP;     // rounds
  static constexpr int P0 = LOGL - LOGP * (R - 1);       // stages in round 0
};

// LDS slot of point j within a line: one padding slot after every P points.
template <int LOGL, int LOGP>
__device__ __forceinline__ u32 pad_idx(u32 j) {
  if constexpr (LOGL > LOGP) return j + (j >> LOGP);
  else return j;
}

// Ordering between the rounds of a line.  The lanes of one line exchange
// points through the line's LDS slots; a line held by at most one wavefront
// (2^(LOGL - LOGP) <= 64 lanes, lines never straddle wavefronts) is private to
// that wavefront, whose LDS accesses execute in order, so the rounds only need
// the compiler kept from moving LDS accesses across the boundary (a
// wavefront-scope fence and barrier) instead of a workgroup barrier.  Longer
// lines, and the end of the last round (the tile's copy-out, or a fused
// product's point-wise step, reads across lines), take __syncthreads.
template <int TPL>
__device__ __forceinline__ void round_sync(bool last) {
  if (TPL <= 64 && !last) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One round of a line: LOGP (or, for round 0, the remainder P0) stages on the
// P points a lane holds, between an LDS load and an LDS store.  In round r the
// lane's point u sits at line index base_j | (u << L0), L0 = LOGL - s0 - LOGP;
// the stages of the round pair the top np bits of u.  Rounds and stages are
// compile-time recursions so every register index is a constant.
template <int W, int LOGL, int LOGP, int DIR, int RIDX, class BF = NativeBfly>
struct Round {
  using S = LineShape<LOGL, LOGP>;
  static constexpr int P = S::P;
  static constexpr int s0 = (RIDX == 0) ? 0 : S::P0 + (RIDX - 1) * LOGP;
  static constexpr int np = (RIDX == 0) ? S::P0 : LOGP;
  static constexpr int L0 = LOGL - s0 - LOGP;

  template <int ST0>
  static __device__ __forceinline__ void stage(Res<W> (&x)[P], u32 base_j, u32 base, const Tw<W>* __restrict__ tw,
                                               const NttParams<W>& p, bool last_inv) {
    constexpr int st = (DIR == DIR_FWD) ? ST0 : (np - 1 - ST0);
    constexpr int s = s0 + st;              // stage index within the line
    constexpr int ib = LOGP - 1 - st;       // bit of u that the stage pairs
    constexpr int ngroups = 1 << st;        // distinct twiddles of the stage
#pragma unroll
    for (int gi = 0; gi < ngroups; ++gi) {
      const u32 j0 = base_j | ((u32)(gi << (ib + 1)) << L0);
      const u32 g = j0 >> (LOGL - s);
      if (DIR == DIR_INV && s == 0 && last_inv) {
#pragma unroll
        for (int lo = 0; lo < (1 << ib); ++lo) {
          const int u = (gi << (ib + 1)) | lo;
          BF::gs_last(x[u], x[u | (1 << ib)], p.ninv, p.ninv_w1, p.M);
        }
      } else {
        const Tw<W> t = load_tw(tw, (base << s) + g);
#pragma unroll
        for (int lo = 0; lo < (1 << ib); ++lo) {
          const int u = (gi << (ib + 1)) | lo;
          if (DIR == DIR_FWD) BF::ct(x[u], x[u | (1 << ib)], t, p.M);
          else BF::gs(x[u], x[u | (1 << ib)], t, p.M);
        }
      }
    }
    if constexpr (ST0 + 1 < np) stage<ST0 + 1>(x, base_j, base, tw, p, last_inv);
  }

  static __device__ __forceinline__ void run(Res<W>* line, u32 tid, u32 base, const Tw<W>* __restrict__ tw,
                                             const NttParams<W>& p, bool last_inv, bool canon, bool last_round) {
    const u32 base_j = ((tid >> L0) << (L0 + LOGP)) | (tid & ((1u << L0) - 1u));
    Res<W> x[P];
#pragma unroll
    for (int u = 0; u < P; ++u) x[u] = line[pad_idx<LOGL, LOGP>(base_j | ((u32)u << L0))];
    stage<0>(x, base_j, base, tw, p, last_inv);
    if (canon) {
#pragma unroll
      for (int u = 0; u < P; ++u) x[u] = BF::canon(x[u], p.M);
    }
#pragma unroll
    for (int u = 0; u < P; ++u) line[pad_idx<LOGL, LOGP>(base_j | ((u32)u << L0))] = x[u];
    round_sync<S::TPL>(last_round);
  }

  // Two points per lane (LOGP == 1): the round is one stage with one twiddle
  // per lane.  Its table index, so that a tile can load the twiddles of all
  // rounds before the first one.
  static __device__ __forceinline__ u32 tw_index(u32 tid, u32 base) {
    static_assert(LOGP == 1, "one stage per round");
    const u32 base_j = ((tid >> L0) << (L0 + LOGP)) | (tid & ((1u << L0) - 1u));
    return (base << s0) + (base_j >> (LOGL - s0));
  }

  // The round with its twiddle already loaded (LOGP == 1).
  static __device__ __forceinline__ void run_loaded(Res<W>* line, u32 tid, const Tw<W>& t, const NttParams<W>& p,
                                                    bool last_inv, bool canon, bool last_round) {
    static_assert(LOGP == 1, "one stage per round");
    const u32 base_j = ((tid >> L0) << (L0 + LOGP)) | (tid & ((1u << L0) - 1u));
    const u32 i0 = pad_idx<LOGL, LOGP>(base_j), i1 = pad_idx<LOGL, LOGP>(base_j | (1u << L0));
    Res<W> x0 = line[i0], x1 = line[i1];
    if (DIR == DIR_INV && s0 == 0 && last_inv) BF::gs_last(x0, x1, p.ninv, p.ninv_w1, p.M);
    else if (DIR == DIR_FWD) BF::ct(x0, x1, t, p.M);
    else BF::gs(x0, x1, t, p.M);
    if (canon) {
      x0 = BF::canon(x0, p.M);
      x1 = BF::canon(x1, p.M);
    }
    line[i0] = x0;
    line[i1] = x1;
    round_sync<S::TPL>(last_round);
  }
};

// The twiddles of every round of a two-point-per-lane line (one per round),
// in round order.  A lane of such a line does little arithmetic per round, so
// a twiddle load issued at the start of each round (after the barrier that
// ends the previous one) leaves its latency exposed once per stage; loading
// them all up front, beside the tile's data loads, pays it once.
template <int W, int LOGL, int DIR, class BF>
struct LineTw {
  Tw<W> t[LOGL];
  template <int RR = 0>
  __device__ __forceinline__ void load(u32 tid, u32 base, const Tw<W>* __restrict__ tw) {
    constexpr int R = (DIR == DIR_FWD) ? RR : (LOGL - 1 - RR);
    t[RR] = load_tw(tw, Round<W, LOGL, 1, DIR, R, BF>::tw_index(tid, base));
    if constexpr (RR + 1 < LOGL) load<RR + 1>(tid, base, tw);
  }
};

// All rounds of a two-point-per-lane line with the twiddles loaded.
template <int W, int LOGL, int DIR, int RR = 0, class BF = NativeBfly>
__device__ __forceinline__ void line_stages_loaded(Res<W>* line, u32 tid, const LineTw<W, LOGL, DIR, BF>& tws,
                                                   const NttParams<W>& p, bool last_inv, bool final_fwd) {
  constexpr int R = (DIR == DIR_FWD) ? RR : (LOGL - 1 - RR);
  Round<W, LOGL, 1, DIR, R, BF>::run_loaded(line, tid, tws.t[RR], p, last_inv,
                                            DIR == DIR_FWD && final_fwd && RR == LOGL - 1, RR == LOGL - 1);
  if constexpr (RR + 1 < LOGL)
    line_stages_loaded<W, LOGL, DIR, RR + 1, BF>(line, tid, tws, p, last_inv, final_fwd);
}

// All rounds of a line held in LDS (forward: rounds 0..R-1; inverse: R-1..0).
// tid: lane index within the line; base: twiddle base (1, or N1 + b for rows);
// last_inv: the line contains the final inverse stage (fold N^-1);
// final_fwd: canonicalize after the last forward stage.
template <int W, int LOGL, int LOGP, int DIR, int RR = 0, class BF = NativeBfly>
__device__ __forceinline__ void line_stages(Res<W>* line, u32 tid, u32 base, const Tw<W>* __restrict__ tw,
                                            const NttParams<W>& p, bool last_inv, bool final_fwd) {
  using S = LineShape<LOGL, LOGP>;
  constexpr int R = (DIR == DIR_FWD) ? RR : (S::R - 1 - RR);
  Round<W, LOGL, LOGP, DIR, R, BF>::run(line, tid, base, tw, p, last_inv,
                                    DIR == DIR_FWD && final_fwd && RR == S::R - 1, RR == S::R - 1);
  if constexpr (RR + 1 < S::R)
    line_stages<W, LOGL, LOGP, DIR, RR + 1, BF>(line, tid, base, tw, p, last_inv, final_fwd);
}

// Number of tiles one launch of a pass covers.
template <int MODE>
__host__ __device__ inline u32 tiles_per_poly(u32 log_n, u32 log_n1, u32 lines) {
  if (MODE == MODE_COL) return (1u << (log_n - log_n1)) / lines;
  if (MODE == MODE_ROW) return (1u << log_n1) / lines;
  return 1;
}

// One tile: device memory -> LDS, the line stages, LDS -> device memory.
// All threads of the workgroup take part (lines * L/P threads); `lds` holds
// lines * NPAD residues.  For MODE_FULL, `tile` indexes groups of `lines`
// transforms; otherwise it indexes (poly, tile-within-poly).
template <int W, int LOGL, int LOGP, int DIR, int MODE, class BF = NativeBfly>
__device__ __forceinline__ void ntt_tile(const NttParams<W>& p, Res<W>* lds, u32 tile) {
  using S = LineShape<LOGL, LOGP>;
  constexpr int L = S::L;
  const u32 lines = p.lines;
  const u32 T = lines * S::TPL;
  const u32 t = threadIdx.x;
  const u32 line_id = t / S::TPL;
  const u32 lane = t % S::TPL;
  const u32 log_n = p.log_n;
  const u64 N = (u64)1 << log_n;
  const u32 log_lines = __builtin_ctz(lines);
  const u32 nelem = lines << LOGL;

  u32 poly;
  u32 c0 = 0, b_lo = 0;
  const u32 log_n1 = p.log_n1, log_n2 = log_n - p.log_n1;
  if (MODE == MODE_FULL) {
    poly = tile;   // group of `lines` transforms
  } else {
    const u32 tiles = tiles_per_poly<MODE>(log_n, log_n1, lines);
    poly = tile / tiles;
    if (MODE == MODE_COL) c0 = (tile % tiles) * lines;
    else b_lo = tile % tiles;
  }
  u32 base = 1;   // twiddle base of the lane's line
  if (MODE == MODE_ROW) base = (1u << log_n1) + line_id * ((1u << log_n1) >> log_lines) + b_lo;
  const bool last_inv = (DIR == DIR_INV) && (MODE != MODE_ROW);
  const bool final_fwd = (DIR == DIR_FWD) && (MODE != MODE_COL);

  // Column and row tiles of two points per lane (the one-transform shapes of
  // two-pass transforms): every round's twiddle is loaded here, in flight
  // with the data loads below.  Measured on MI355X, batch-1 forward + inverse:
  // two-word 2^16 23.4 -> 22.0 us, 2^17 27.1 -> 25.4 us.  Single-workgroup
  // transforms of 2^11 points were slower this way (15.2 -> 16.0 us), and
  // four-word twiddles would take 16 registers per round.
  constexpr bool kLoadTw = LOGP == 1 && W <= 4 && MODE != MODE_FULL;
  LineTw<W, LOGL, DIR, BF> tws;
  if constexpr (kLoadTw) tws.load(lane, base, p.tw);

  // ---- device memory -> LDS ----
  // lines * L/P threads move lines * L elements: exactly P each, no guard
  constexpr int P = S::P;
  const auto all = [](u32) { return true; };
  if (MODE == MODE_FULL) {
    copy_staged<W, P>(
        t, T, [&](u32 e) { return e < nelem && (u64)poly * lines + (e >> LOGL) < p.batch; },
        [&](u32 e) { return ResIO<W>::load(p.src + ((u64)poly * lines + (e >> LOGL)) * N + (e & (L - 1))); },
        [&](u32 e, const Res<W>& v) {
          const u32 j = e & (L - 1);
          const u32 dj = (DIR == DIR_INV && p.permute) ? brev(j, LOGL) : j;
          lds[(e >> LOGL) * S::NPAD + pad_idx<LOGL, LOGP>(dj)] = v;
        });
  } else if (MODE == MODE_COL) {
    const u64 N2 = (u64)1 << log_n2;
    copy_staged<W, P>(
        t, T, all,
        [&](u32 e) { return ResIO<W>::load(p.src + (u64)poly * N + (e >> log_lines) * N2 + c0 + (e & (lines - 1))); },
        [&](u32 e, const Res<W>& v) { lds[(e & (lines - 1)) * S::NPAD + pad_idx<LOGL, LOGP>(e >> log_lines)] = v; });
  } else {
    const u32 n1_over_g = (1u << log_n1) >> log_lines;
    if (DIR == DIR_INV && p.permute) {
      // natural-order input: run of G residues at k = l'*N1 + bitrev(b_lo)*G + jj
      const u32 col = brev(b_lo, log_n1 - log_lines) << log_lines;
      copy_staged<W, P>(
          t, T, all,
          [&](u32 e) {
            return ResIO<W>::load(p.src + (u64)poly * N + ((u64)(e >> log_lines) << log_n1) + col + (e & (lines - 1)));
          },
          [&](u32 e, const Res<W>& v) {
            lds[brev(e & (lines - 1), log_lines) * S::NPAD + pad_idx<LOGL, LOGP>(brev(e >> log_lines, LOGL))] = v;
          });
    } else {
      copy_staged<W, P>(
          t, T, all,
          [&](u32 e) {
            const u32 b = (e >> LOGL) * n1_over_g + b_lo;
            return ResIO<W>::load(p.src + (u64)poly * N + ((u64)b << LOGL) + (e & (L - 1)));
          },
          [&](u32 e, const Res<W>& v) { lds[(e >> LOGL) * S::NPAD + pad_idx<LOGL, LOGP>(e & (L - 1))] = v; });
    }
  }
  __syncthreads();

  // ---- stages ----
  if constexpr (kLoadTw)
    line_stages_loaded<W, LOGL, DIR, 0, BF>(lds + line_id * S::NPAD, lane, tws, p, last_inv, final_fwd);
  else
    line_stages<W, LOGL, LOGP, DIR, 0, BF>(lds + line_id * S::NPAD, lane, base, p.tw, p, last_inv, final_fwd);

  // ---- LDS -> device memory ----
  if (MODE == MODE_FULL) {
    copy_staged<W, P>(
        t, T, [&](u32 e) { return e < nelem && (u64)poly * lines + (e >> LOGL) < p.batch; },
        [&](u32 e) {
          const u32 j = e & (L - 1);
          const u32 sj = (DIR == DIR_FWD && p.permute) ? brev(j, LOGL) : j;
          return lds[(e >> LOGL) * S::NPAD + pad_idx<LOGL, LOGP>(sj)];
        },
        [&](u32 e, const Res<W>& v) {
          ResIO<W>::store(p.dst + ((u64)poly * lines + (e >> LOGL)) * N + (e & (L - 1)), v);
        });
  } else if (MODE == MODE_COL) {
    const u64 N2 = (u64)1 << log_n2;
    copy_staged<W, P>(
        t, T, all,
        [&](u32 e) { return lds[(e & (lines - 1)) * S::NPAD + pad_idx<LOGL, LOGP>(e >> log_lines)]; },
        [&](u32 e, const Res<W>& v) {
          ResIO<W>::store(p.dst + (u64)poly * N + (e >> log_lines) * N2 + c0 + (e & (lines - 1)), v);
        });
  } else {
    const u32 n1_over_g = (1u << log_n1) >> log_lines;
    if (DIR == DIR_FWD && p.permute) {
      const u32 col = brev(b_lo, log_n1 - log_lines) << log_lines;
      copy_staged<W, P>(
          t, T, all,
          [&](u32 e) {
            return lds[brev(e & (lines - 1), log_lines) * S::NPAD + pad_idx<LOGL, LOGP>(brev(e >> log_lines, LOGL))];
          },
          [&](u32 e, const Res<W>& v) {
            ResIO<W>::store(p.dst + (u64)poly * N + ((u64)(e >> log_lines) << log_n1) + col + (e & (lines - 1)), v);
          });
    } else {
      copy_staged<W, P>(
          t, T, all,
          [&](u32 e) { return lds[(e >> LOGL) * S::NPAD + pad_idx<LOGL, LOGP>(e & (L - 1))]; },
          [&](u32 e, const Res<W>& v) {
            const u32 b = (e >> LOGL) * n1_over_g + b_lo;
            ResIO<W>::store(p.dst + (u64)poly * N + ((u64)b << LOGL) + (e & (L - 1)), v);
          });
    }
  }
}

// Largest workgroup a tile kernel of this shape is compiled for.
template <int LOGL, int LOGP>
constexpr int max_threads() {
  constexpr int tpl = 1 << (LOGL - LOGP);
  return tpl > 256 ? (tpl > 1024 ? 1024 : tpl) : 256;
}

// Largest points-per-lane exponent and single-workgroup transform per width:
// four-word residues take 8 registers each, so their lanes hold at most 4
// points, and a single-workgroup transform at most 2^11 of them (LDS).
__host__ __device__ constexpr int max_logp(int W) { return W == 8 ? 2 : 4; }
__host__ __device__ constexpr int max_full_log(int W) { return W == 8 ? 11 : (W == 4 ? 12 : 13); }

// Kernel shapes that are instantiated: full transforms of 2^1..2^12 points
// (2^13 for one-word moduli, 2^11 for four-word); column / row lines of
// 2^3..2^9 points; points per lane 2^1..2^max_logp with at most 1024 lanes
// per line.
template <int W, int MODE>
constexpr bool shape_ok(int logl, int logp) {
  if (logp < 1 || logp > max_logp(W) || logp > logl) return false;
  if (logl - logp > 10) return false;
  if (MODE == MODE_FULL) return logl >= 1 && logl <= max_full_log(W);
  return logl >= 3 && logl <= 9;
}

extern "C++" {
template <int W, int DIR>
hipError_t launch_ntt(int mode, u32 logl, u32 logp, const NttParams<W>& p, u32 blocks, hipStream_t s);
}

// Dynamic LDS bytes of a tile.
template <int W>
inline size_t tile_lds_bytes(u32 logl, u32 logp, u32 lines) {
  const u32 L = 1u << logl, P = 1u << logp;
  const u32 npad = ((logl > logp) ? L + L / P : L) + 1;
  return (size_t)lines * npad * sizeof(Res<W>);
}

}  // namespace mw
