// Negacyclic NTT / INTT over Z_q[X]/(X^N + 1) for gfx950.
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
//   * N <= 2^12 (2^13 for one-word moduli): one line per transform, the whole
//     transform in one workgroup ("full" tiles);
//   * larger N: N = N1 * N2 and two passes over HBM.  The first log N1
//     Cooley-Tukey stages only pair elements in the same residue class mod N2
//     (columns of stride N2) and use the table entries below N1, so a column
//     is an N1-point line with twiddle base 1.  The remaining log N2 stages act
//     within contiguous rows of N2 elements; row b is an N2-point line whose
//     local stage m' uses tw[m' * (N1 + b) + g].  No transpose and no extra
//     twiddle pass are needed.  The inverse runs the rows first, then the
//     columns.
//   * natural-order output of the forward transform: row b, local index l
//     holds A at k = bitrev(l)*N1 + bitrev(b).  A row tile takes G rows
//     b = j*(N1/G) + b_lo, whose outputs land in runs of G consecutive
//     residues, so the permuted store (and the inverse's permuted load) is
//     coalesced in G*16-byte segments.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <vector>

#include "mw_arith.h"
#include "mw_common.h"

namespace mw {

template <int W>
struct Tw {
  u32 w[W];
  u32 ws[W];
};

template <int W>
__device__ __forceinline__ Tw<W> load_tw(const Tw<W>* t, u32 idx) {
  Tw<W> r;
  if constexpr (W == 4) {
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
  u32 batch;
  u32 permute;           // 1: natural order at the HBM side of this pass
};

// Forward (Cooley-Tukey) butterfly on [0, 16q) values.
template <int W>
__device__ __forceinline__ void ct_bfly(Res<W>& X, Res<W>& Y, const Tw<W>& t, const Modulus<W>& M) {
  Res<W> T = shoup_mul(Y, t.w, t.ws, M);   // [0, 6q)
  Res<W> Xr = csub(X, M.q8);               // [0, 8q)
  X = add(Xr, T);                          // [0, 14q)
  Res<W> D = add(Xr, M.q8);                // [8q, 16q)
  u32 b;
  Y = sub(D, T, b);                        // (2q, 16q)
}

// Inverse (Gentleman-Sande) butterfly on [0, 8q) values.
template <int W>
__device__ __forceinline__ void gs_bfly(Res<W>& X, Res<W>& Y, const Tw<W>& t, const Modulus<W>& M) {
  Res<W> S = csub(add(X, Y), M.q8);        // [0, 8q)
  Res<W> D = add(X, M.q8);
  u32 b;
  D = sub(D, Y, b);                        // (0, 16q)
  Y = shoup_mul(D, t.w, t.ws, M);          // [0, 6q)
  X = S;
}

// Last inverse stage with N^-1 folded in; outputs canonical.
template <int W>
__device__ __forceinline__ void gs_bfly_last(Res<W>& X, Res<W>& Y, const Tw<W>& ninv, const Tw<W>& ninv_w1,
                                             const Modulus<W>& M) {
  Res<W> S = add(X, Y);                    // [0, 16q) < 2^(32W)
  Res<W> D = add(X, M.q8);
  u32 b;
  D = sub(D, Y, b);                        // (0, 16q)
  Res<W> x = shoup_mul(S, ninv.w, ninv.ws, M);     // [0, 6q)
  Res<W> y = shoup_mul(D, ninv_w1.w, ninv_w1.ws, M);
  x = csub(csub(csub(x, M.q4), M.q2), M.q);
  y = csub(csub(csub(y, M.q4), M.q2), M.q);
  X = x;
  Y = y;
}

template <int W>
__device__ __forceinline__ Res<W> canon16(const Res<W>& x, const Modulus<W>& M) {
  return csub(csub(csub(csub(x, M.q8), M.q4), M.q2), M.q);
}

__device__ __forceinline__ u32 brev(u32 x, u32 bits) {
  return bits ? (__builtin_bitreverse32(x) >> (32 - bits)) : 0u;
}

// LDS slot of point j within a line: one padding slot after every P points.
template <int LOGL, int LOGP>
__device__ __forceinline__ u32 pad_idx(u32 j) {
  if constexpr (LOGL > LOGP) return j + (j >> LOGP);
  else return j;
}

template <int LOGL, int LOGP>
struct LineShape {
  static constexpr int L = 1 << LOGL;
  static constexpr int P = 1 << LOGP;
  static constexpr int TPL = L / P;                      // lanes per line
  static constexpr int NPAD = (LOGL > LOGP) ? L + L / P : L;
  static constexpr int R = (LOGL + LOGP - 1) / LOGP;     // rounds
  static constexpr int P0 = LOGL - LOGP * (R - 1);       // stages in round 0
};

// One round of a line: LOGP (or, for round 0, the remainder P0) stages on the
// P points a lane holds, between an LDS load and an LDS store.  In round r the
// lane's point u sits at line index base_j | (u << L0), L0 = LOGL - s0 - LOGP;
// the stages of the round pair the top np bits of u.  Rounds and stages are
// compile-time recursions so every register index is a constant.
template <int W, int LOGL, int LOGP, int DIR, int RIDX>
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
          gs_bfly_last(x[u], x[u | (1 << ib)], p.ninv, p.ninv_w1, p.M);
        }
      } else {
        const Tw<W> t = load_tw(tw, (base << s) + g);
#pragma unroll
        for (int lo = 0; lo < (1 << ib); ++lo) {
          const int u = (gi << (ib + 1)) | lo;
          if (DIR == DIR_FWD) ct_bfly(x[u], x[u | (1 << ib)], t, p.M);
          else gs_bfly(x[u], x[u | (1 << ib)], t, p.M);
        }
      }
    }
    if constexpr (ST0 + 1 < np) stage<ST0 + 1>(x, base_j, base, tw, p, last_inv);
  }

  static __device__ __forceinline__ void run(Res<W>* line, u32 tid, u32 base, const Tw<W>* __restrict__ tw,
                                             const NttParams<W>& p, bool last_inv, bool canon) {
    const u32 base_j = ((tid >> L0) << (L0 + LOGP)) | (tid & ((1u << L0) - 1u));
    Res<W> x[P];
#pragma unroll
    for (int u = 0; u < P; ++u) x[u] = line[pad_idx<LOGL, LOGP>(base_j | ((u32)u << L0))];
    stage<0>(x, base_j, base, tw, p, last_inv);
    if (canon) {
#pragma unroll
      for (int u = 0; u < P; ++u) x[u] = canon16(x[u], p.M);
    }
#pragma unroll
    for (int u = 0; u < P; ++u) line[pad_idx<LOGL, LOGP>(base_j | ((u32)u << L0))] = x[u];
    __syncthreads();
  }
};

// All rounds of a line held in LDS (forward: rounds 0..R-1; inverse: R-1..0).
// tid: lane index within the line; base: twiddle base (1, or N1 + b for rows);
// last_inv: the line contains the final inverse stage (fold N^-1);
// final_fwd: canonicalize after the last forward stage.
template <int W, int LOGL, int LOGP, int DIR, int RR = 0>
__device__ __forceinline__ void line_stages(Res<W>* line, u32 tid, u32 base, const Tw<W>* __restrict__ tw,
                                            const NttParams<W>& p, bool last_inv, bool final_fwd) {
  using S = LineShape<LOGL, LOGP>;
  constexpr int R = (DIR == DIR_FWD) ? RR : (S::R - 1 - RR);
  Round<W, LOGL, LOGP, DIR, R>::run(line, tid, base, tw, p, last_inv,
                                    DIR == DIR_FWD && final_fwd && RR == S::R - 1);
  if constexpr (RR + 1 < S::R) line_stages<W, LOGL, LOGP, DIR, RR + 1>(line, tid, base, tw, p, last_inv, final_fwd);
}

template <int W, int LOGL, int LOGP, int LINES, int DIR, int MODE>
__global__ __launch_bounds__(LINES*(1 << (LOGL - LOGP))) void ntt_kernel(NttParams<W> p) {
  using S = LineShape<LOGL, LOGP>;
  constexpr int T = LINES * S::TPL;
  constexpr int L = S::L;
  __shared__ Res<W> lds[LINES * S::NPAD];

  const u32 t = threadIdx.x;
  const u32 line_id = t / S::TPL;
  const u32 lane = t % S::TPL;
  const u32 log_n = p.log_n;
  const u64 N = (u64)1 << log_n;

  u32 poly;
  u32 c0 = 0, b_lo = 0, log_g = 0, log_n1 = p.log_n1, log_n2 = log_n - p.log_n1;
  if (MODE == MODE_FULL) {
    poly = blockIdx.x;   // LINES polys per block
  } else if (MODE == MODE_COL) {
    const u32 tiles = (1u << log_n2) / LINES;
    poly = blockIdx.x / tiles;
    c0 = (blockIdx.x % tiles) * LINES;
  } else {
    const u32 tiles = (1u << log_n1) / LINES;
    poly = blockIdx.x / tiles;
    b_lo = blockIdx.x % tiles;
    log_g = __builtin_ctz((u32)LINES);
  }

  // ---- HBM -> LDS ----
  if (MODE == MODE_FULL) {
#pragma unroll
    for (int k = 0; k < LINES * L / T; ++k) {
      const u32 e = t + k * T;
      const u32 ln = e >> LOGL, j = e & (L - 1);
      const u64 pl = (u64)poly * LINES + ln;
      if (pl < p.batch) {
        const u32 dj = (DIR == DIR_INV && p.permute) ? brev(j, LOGL) : j;
        lds[ln * S::NPAD + pad_idx<LOGL, LOGP>(dj)] = ResIO<W>::load(p.src + pl * N + j);
      }
    }
  } else if (MODE == MODE_COL) {
    const u64 N2 = (u64)1 << log_n2;
#pragma unroll
    for (int k = 0; k < LINES * L / T; ++k) {
      const u32 e = t + k * T;
      const u32 r = e / LINES, c = e % LINES;
      lds[c * S::NPAD + pad_idx<LOGL, LOGP>(r)] = ResIO<W>::load(p.src + (u64)poly * N + r * N2 + c0 + c);
    }
  } else {
    const u32 n1_over_g = (1u << log_n1) >> log_g;
    if (DIR == DIR_INV && p.permute) {
      // natural-order input: run of G residues at k = l'*N1 + bitrev(b_lo)*G + jj
      const u32 col = brev(b_lo, log_n1 - log_g) << log_g;
#pragma unroll
      for (int k = 0; k < LINES * L / T; ++k) {
        const u32 e = t + k * T;
        const u32 lp = e / LINES, jj = e % LINES;
        const u64 src = (u64)poly * N + ((u64)lp << log_n1) + col + jj;
        lds[brev(jj, log_g) * S::NPAD + pad_idx<LOGL, LOGP>(brev(lp, LOGL))] = ResIO<W>::load(p.src + src);
      }
    } else {
#pragma unroll
      for (int k = 0; k < LINES * L / T; ++k) {
        const u32 e = t + k * T;
        const u32 j = e >> LOGL, l = e & (L - 1);
        const u32 b = j * n1_over_g + b_lo;
        lds[j * S::NPAD + pad_idx<LOGL, LOGP>(l)] = ResIO<W>::load(p.src + (u64)poly * N + ((u64)b << LOGL) + l);
      }
    }
  }
  __syncthreads();

  // ---- stages ----
  u32 base = 1;
  if (MODE == MODE_ROW) base = (1u << log_n1) + line_id * ((1u << log_n1) >> log_g) + b_lo;
  const bool last_inv = (DIR == DIR_INV) && (MODE != MODE_ROW);
  const bool final_fwd = (DIR == DIR_FWD) && (MODE != MODE_COL);
  line_stages<W, LOGL, LOGP, DIR>(lds + line_id * S::NPAD, lane, base, p.tw, p, last_inv, final_fwd);

  // ---- LDS -> HBM ----
  if (MODE == MODE_FULL) {
#pragma unroll
    for (int k = 0; k < LINES * L / T; ++k) {
      const u32 e = t + k * T;
      const u32 ln = e >> LOGL, j = e & (L - 1);
      const u64 pl = (u64)poly * LINES + ln;
      if (pl < p.batch) {
        const u32 sj = (DIR == DIR_FWD && p.permute) ? brev(j, LOGL) : j;
        ResIO<W>::store(p.dst + pl * N + j, lds[ln * S::NPAD + pad_idx<LOGL, LOGP>(sj)]);
      }
    }
  } else if (MODE == MODE_COL) {
    const u64 N2 = (u64)1 << log_n2;
#pragma unroll
    for (int k = 0; k < LINES * L / T; ++k) {
      const u32 e = t + k * T;
      const u32 r = e / LINES, c = e % LINES;
      ResIO<W>::store(p.dst + (u64)poly * N + r * N2 + c0 + c, lds[c * S::NPAD + pad_idx<LOGL, LOGP>(r)]);
    }
  } else {
    const u32 n1_over_g = (1u << log_n1) >> log_g;
    if (DIR == DIR_FWD && p.permute) {
      const u32 col = brev(b_lo, log_n1 - log_g) << log_g;
#pragma unroll
      for (int k = 0; k < LINES * L / T; ++k) {
        const u32 e = t + k * T;
        const u32 lp = e / LINES, jj = e % LINES;
        const u64 dst = (u64)poly * N + ((u64)lp << log_n1) + col + jj;
        ResIO<W>::store(p.dst + dst, lds[brev(jj, log_g) * S::NPAD + pad_idx<LOGL, LOGP>(brev(lp, LOGL))]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < LINES * L / T; ++k) {
        const u32 e = t + k * T;
        const u32 j = e >> LOGL, l = e & (L - 1);
        const u32 b = j * n1_over_g + b_lo;
        ResIO<W>::store(p.dst + (u64)poly * N + ((u64)b << LOGL) + l, lds[j * S::NPAD + pad_idx<LOGL, LOGP>(l)]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launch configuration
// ---------------------------------------------------------------------------
constexpr int kLogP = 3;           // 8 points per lane
constexpr int kColLines = 8;       // columns per column tile
constexpr int kRowLines = 8;       // rows per row tile
constexpr int kMaxFullLog4 = 12;   // largest single-workgroup transform, two-word moduli
constexpr int kMaxFullLog2 = 13;   // one-word moduli

template <int LOGL>
constexpr int full_lines() {
  // aim at 256 lanes per block, at least one line
  constexpr int lp = LOGL < kLogP ? LOGL : kLogP;
  constexpr int tpl = 1 << (LOGL - lp);
  return tpl >= 256 ? 1 : 256 / tpl;
}

template <int W, int LOGL, int DIR, int MODE>
static hipError_t launch_one(const NttParams<W>& p, u32 blocks, hipStream_t s) {
  constexpr int LOGP = LOGL < kLogP ? LOGL : kLogP;
  constexpr int LINES = (MODE == MODE_FULL) ? full_lines<LOGL>() : (MODE == MODE_COL ? kColLines : kRowLines);
  constexpr int T = LINES * (1 << (LOGL - LOGP));
  hipLaunchKernelGGL((ntt_kernel<W, LOGL, LOGP, LINES, DIR, MODE>), dim3(blocks), dim3(T), 0, s, p);
  return hipGetLastError();
}

// Line lengths instantiated per mode: single-workgroup transforms of 2^1 up to
// 2^12 points (2^13 for one-word moduli); column / row lines of 2^3 .. 2^9.
template <int W, int MODE>
constexpr bool instantiated(int logl) {
  if (MODE == MODE_FULL) return logl >= 1 && logl <= (W == 4 ? kMaxFullLog4 : kMaxFullLog2);
  return logl >= 3 && logl <= 9;
}

template <int W, int DIR, int MODE>
static hipError_t launch_by_log(u32 logl, const NttParams<W>& p, u32 blocks, hipStream_t s) {
  switch (logl) {
#define MW_CASE(LG)                                                                   \
  case LG:                                                                            \
    if constexpr (instantiated<W, MODE>(LG)) return launch_one<W, LG, DIR, MODE>(p, blocks, s); \
    return hipErrorInvalidValue;
    MW_CASE(1) MW_CASE(2) MW_CASE(3) MW_CASE(4) MW_CASE(5) MW_CASE(6) MW_CASE(7) MW_CASE(8) MW_CASE(9)
    MW_CASE(10) MW_CASE(11) MW_CASE(12) MW_CASE(13)
#undef MW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <int W>
static u32 full_lines_for(u32 logl) {
  switch (logl) {
#define MW_CASE(LG) \
  case LG:          \
    return full_lines<LG>();
    MW_CASE(1) MW_CASE(2) MW_CASE(3) MW_CASE(4) MW_CASE(5) MW_CASE(6) MW_CASE(7) MW_CASE(8) MW_CASE(9)
    MW_CASE(10) MW_CASE(11) MW_CASE(12) MW_CASE(13)
#undef MW_CASE
    default:
      return 1;
  }
}

}  // namespace mw

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
using namespace mw;

struct ntt_plan_s {
  uint32_t log2n = 0, limbs = 0, flags = 0;
  uint32_t log_n1 = 0;        // 0: single-tile transform
  uint64_t q[2] = {0, 0};
  uint64_t psi[2] = {0, 0};
  int device = 0;
  void* d_tw_fwd = nullptr;   // N entries of {w, w'}
  void* d_tw_inv = nullptr;
  void* d_scratch = nullptr;  // two-pass intermediate
  uint32_t scratch_polys = 0;
  Modulus<4> M4;
  Modulus<2> M2;
  Tw<4> ninv4, last4;
  Tw<2> ninv2, last2;
};

namespace {

template <int W>
void fill_tw(Tw<W>& t, mwhost::u128 w, mwhost::u128 q) {
  put_words<W>(w, t.w);
  put_words<W>(mwhost::shoup(w, q, 32 * W), t.ws);
}

template <int W>
int build_tables(ntt_plan_s* P, mwhost::u128 q, mwhost::u128 psi) {
  const uint32_t n = 1u << P->log2n;
  const int logn = (int)P->log2n;
  std::vector<Tw<W>> fwd(n), inv(n);
  mwhost::u128 psi_inv = mwhost::invmod(psi, q);
  // powers psi^e and psi^-e for e < N, then place at bit-reversed positions
  std::vector<mwhost::u128> pw(n), pwi(n);
  pw[0] = 1;
  pwi[0] = 1;
  for (uint32_t e = 1; e < n; ++e) {
    pw[e] = mwhost::mulmod(pw[e - 1], psi, q);
    pwi[e] = mwhost::mulmod(pwi[e - 1], psi_inv, q);
  }
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t e = mwhost::bitrev(i, logn);
    fill_tw<W>(fwd[i], pw[e], q);
    fill_tw<W>(inv[i], pwi[e], q);
  }
  mwhost::u128 ninv = mwhost::invmod((mwhost::u128)n, q);
  mwhost::u128 w1 = (n >= 2) ? pwi[mwhost::bitrev(1, logn)] : 1;
  Tw<W> tn, tl;
  fill_tw<W>(tn, ninv, q);
  fill_tw<W>(tl, mwhost::mulmod(w1, ninv, q), q);
  if constexpr (W == 4) {
    P->ninv4 = tn;
    P->last4 = tl;
  } else {
    P->ninv2 = tn;
    P->last2 = tl;
  }
  size_t bytes = sizeof(Tw<W>) * n;
  if (hipMalloc(&P->d_tw_fwd, bytes) != hipSuccess) return MW_ENOMEM;
  if (hipMalloc(&P->d_tw_inv, bytes) != hipSuccess) return MW_ENOMEM;
  if (hipMemcpy(P->d_tw_fwd, fwd.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return MW_EDEVICE;
  if (hipMemcpy(P->d_tw_inv, inv.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return MW_EDEVICE;
  return MW_OK;
}

void free_plan(ntt_plan_s* P) {
  if (!P) return;
  if (P->d_tw_fwd) (void)hipFree(P->d_tw_fwd);
  if (P->d_tw_inv) (void)hipFree(P->d_tw_inv);
  if (P->d_scratch) (void)hipFree(P->d_scratch);
  delete P;
}

// Scratch for the two-pass transforms: up to 64 MiB, at least one polynomial.
constexpr size_t kScratchBytes = size_t(64) << 20;

template <int W>
int run_transform(ntt_plan_s* P, void* d_out, const void* d_in, uint32_t batch, int dir, hipStream_t s) {
  NttParams<W> p = {};
  p.tw = reinterpret_cast<const Tw<W>*>(dir == DIR_FWD ? P->d_tw_fwd : P->d_tw_inv);
  if constexpr (W == 4) {
    p.M = P->M4;
    p.ninv = P->ninv4;
    p.ninv_w1 = P->last4;
  } else {
    p.M = P->M2;
    p.ninv = P->ninv2;
    p.ninv_w1 = P->last2;
  }
  p.log_n = P->log2n;
  p.log_n1 = P->log_n1;
  const uint64_t N = 1ull << P->log2n;
  hipError_t e = hipSuccess;
  if (P->log_n1 == 0) {
    p.src = reinterpret_cast<const Res<W>*>(d_in);
    p.dst = reinterpret_cast<Res<W>*>(d_out);
    p.batch = batch;
    p.permute = dir == DIR_FWD ? !(P->flags & NTT_BITREV_OUT) : !(P->flags & NTT_BITREV_IN);
    const u32 lines = full_lines_for<W>(P->log2n);
    const u32 blocks = (batch + lines - 1) / lines;
    e = dir == DIR_FWD ? launch_by_log<W, DIR_FWD, MODE_FULL>(P->log2n, p, blocks, s)
                       : launch_by_log<W, DIR_INV, MODE_FULL>(P->log2n, p, blocks, s);
    return e == hipSuccess ? MW_OK : MW_EDEVICE;
  }
  const u32 log_n1 = P->log_n1, log_n2 = P->log2n - P->log_n1;
  const u32 col_tiles = (1u << log_n2) / kColLines;
  const u32 row_tiles = (1u << log_n1) / kRowLines;
  const uint32_t chunk = P->scratch_polys;
  for (uint32_t b0 = 0; b0 < batch; b0 += chunk) {
    const uint32_t nb = (batch - b0 < chunk) ? batch - b0 : chunk;
    const Res<W>* in = reinterpret_cast<const Res<W>*>(d_in) + (uint64_t)b0 * N;
    Res<W>* out = reinterpret_cast<Res<W>*>(d_out) + (uint64_t)b0 * N;
    Res<W>* scr = reinterpret_cast<Res<W>*>(P->d_scratch);
    p.batch = nb;
    if (dir == DIR_FWD) {
      p.src = in;
      p.dst = scr;
      p.permute = 0;
      e = launch_by_log<W, DIR_FWD, MODE_COL>(log_n1, p, nb * col_tiles, s);
      if (e != hipSuccess) break;
      p.src = scr;
      p.dst = out;
      p.permute = !(P->flags & NTT_BITREV_OUT);
      e = launch_by_log<W, DIR_FWD, MODE_ROW>(log_n2, p, nb * row_tiles, s);
    } else {
      p.src = in;
      p.dst = scr;
      p.permute = !(P->flags & NTT_BITREV_IN);
      e = launch_by_log<W, DIR_INV, MODE_ROW>(log_n2, p, nb * row_tiles, s);
      if (e != hipSuccess) break;
      p.src = scr;
      p.dst = out;
      p.permute = 0;
      e = launch_by_log<W, DIR_INV, MODE_COL>(log_n1, p, nb * col_tiles, s);
    }
    if (e != hipSuccess) break;
  }
  return e == hipSuccess ? MW_OK : MW_EDEVICE;
}

int transform(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream, int dir) {
  if (!plan) return MW_EINVAL;
  if (batch == 0) return MW_OK;
  if (!d_out || !d_in) return MW_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return plan->limbs == 2 ? run_transform<4>(plan, d_out, d_in, batch, dir, s)
                          : run_transform<2>(plan, d_out, d_in, batch, dir, s);
}

// Default two-pass split: N1 = 2^floor(log N / 2) rows, N2 = N / N1.
uint32_t default_split(uint32_t log2n, uint32_t limbs) {
  const uint32_t max_full = limbs == 2 ? kMaxFullLog4 : kMaxFullLog2;
  if (log2n <= max_full) return 0;
  return log2n / 2;
}

}  // namespace

extern "C" int ntt_plan(ntt_plan_t* out, uint32_t log2n, const uint64_t* q, uint32_t limbs,
                        const uint64_t* psi, uint32_t flags) {
  if (!out) return MW_EINVAL;
  *out = nullptr;
  if (flags & ~(NTT_BITREV_OUT | NTT_BITREV_IN)) return MW_EINVAL;
  if (log2n < 1 || log2n > 17) return MW_ESIZE;
  int st = check_modulus(q, limbs, false);
  if (st != MW_OK) return st;
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  const uint32_t n = 1u << log2n;
  if ((Q - 1) % (2 * (mwhost::u128)n) != 0) return MW_EMODULUS;
  mwhost::u128 root;
  if (psi) {
    root = mwhost::from_words(psi, limbs);
    if (root == 0 || root >= Q || mwhost::powmod(root, n, Q) != Q - 1) return MW_EROOT;
  } else {
    root = mwhost::canonical_root(Q, n);
    if (root == 0) return MW_EROOT;
  }
  ntt_plan_s* P = new (std::nothrow) ntt_plan_s();
  if (!P) return MW_ENOMEM;
  P->log2n = log2n;
  P->limbs = limbs;
  P->flags = flags;
  P->q[0] = q[0];
  P->q[1] = limbs > 1 ? q[1] : 0;
  mwhost::to_words(root, P->psi, limbs);
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return MW_EDEVICE;
  }
  if (limbs == 2) make_modulus<4>(q, limbs, P->M4);
  else make_modulus<2>(q, limbs, P->M2);
  st = limbs == 2 ? build_tables<4>(P, Q, root) : build_tables<2>(P, Q, root);
  if (st != MW_OK) {
    free_plan(P);
    return st;
  }
  P->log_n1 = default_split(log2n, limbs);
  if (P->log_n1) {
    const size_t poly_bytes = (size_t)8 * limbs * n;
    size_t polys = kScratchBytes / poly_bytes;
    if (polys < 1) polys = 1;
    P->scratch_polys = (uint32_t)polys;
    if (hipMalloc(&P->d_scratch, polys * poly_bytes) != hipSuccess) {
      free_plan(P);
      return MW_ENOMEM;
    }
  }
  *out = P;
  return MW_OK;
}

extern "C" int ntt_plan_set_split(ntt_plan_t plan, uint32_t log_n1) {
  if (!plan) return MW_EINVAL;
  const uint32_t max_full = plan->limbs == 2 ? kMaxFullLog4 : kMaxFullLog2;
  if (log_n1 == 0) {
    if (plan->log2n > max_full) return MW_ESIZE;
    plan->log_n1 = 0;
    return MW_OK;
  }
  const uint32_t log_n2 = plan->log2n > log_n1 ? plan->log2n - log_n1 : 0;
  if (log_n1 < 3 || log_n1 > 9 || log_n2 < 3 || log_n2 > 9) return MW_ESIZE;
  if (!plan->d_scratch) {
    const size_t poly_bytes = (size_t)8 * plan->limbs << plan->log2n;
    size_t polys = kScratchBytes / poly_bytes;
    if (polys < 1) polys = 1;
    if (hipMalloc(&plan->d_scratch, polys * poly_bytes) != hipSuccess) return MW_ENOMEM;
    plan->scratch_polys = (uint32_t)polys;
  }
  plan->log_n1 = log_n1;
  return MW_OK;
}

extern "C" int ntt_plan_get_split(ntt_plan_t plan, uint32_t* log_n1) {
  if (!plan || !log_n1) return MW_EINVAL;
  *log_n1 = plan->log_n1;
  return MW_OK;
}

extern "C" int ntt_plan_destroy(ntt_plan_t plan) {
  if (!plan) return MW_EINVAL;
  (void)hipDeviceSynchronize();
  free_plan(plan);
  return MW_OK;
}

extern "C" int ntt_plan_root(ntt_plan_t plan, uint64_t* psi_out) {
  if (!plan || !psi_out) return MW_EINVAL;
  psi_out[0] = plan->psi[0];
  if (plan->limbs > 1) psi_out[1] = plan->psi[1];
  return MW_OK;
}

extern "C" int ntt_forward(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream) {
  return transform(plan, d_out, d_in, batch, stream, DIR_FWD);
}

extern "C" int ntt_inverse(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream) {
  return transform(plan, d_out, d_in, batch, stream, DIR_INV);
}
