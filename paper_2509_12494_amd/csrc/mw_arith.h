// Multi-word modular arithmetic for gfx950 (CDNA4) vector lanes.
//
// A residue of an l-bit modulus is held in W little-endian 32-bit words per
// lane: W = 2 for q < 2^60 (one 64-bit limb), W = 4 for q < 2^124 (two 64-bit
// limbs), W = 8 for q < 2^252 (four 64-bit limbs: the wider fields the paper
// names as the next step beyond 128-bit arithmetic, Discussion, larger
// bit-widths).  The paper's double-word arithmetic (Background, double-word
// arithmetic: add with carry, sub with borrow, the schoolbook product of
// Eq. muls) maps onto CDNA4 vector instructions as follows:
//   * word product      -> v_mad_u64_u32 (32x32+64 -> 64, with carry-out mask)
//   * add with carry    -> v_add_co_u32 / v_addc_co_u32 (carry in a lane mask)
//   * sub with borrow   -> v_sub_co_u32 / v_subb_co_u32
//   * masked select     -> v_cndmask_b32 on the borrow mask
// which is the per-lane carry support the paper's MQX extension proposes for
// AVX-512 (Table tab:mqx).  On gfx950 the 32-bit multiplies issue at the same
// rate as the carry adds, so the cost of a mul-mod is its instruction count.
//
// Reductions:
//   * Shoup multiplication by a constant w with precomputed
//     w' = floor(w * 2^(32W) / q) (twiddle factors, the axpy scalar).  The
//     quotient estimate uses only the partial products of columns >= W-1 of
//     x*w' (columns 0..W-2 are dropped; for W = 8 columns >= W-2), which
//     under-estimates the exact Shoup quotient by at most 4 (W=4) or 1 (W=2,
//     W=8); the result x*w - Q*q is then in [0, 6q) for any x < 2^(32W).
//   * Barrett reduction (Background, modular arithmetic, Eq. barrett) for a
//     product of two variables.  The reduction holds for any modulus; to keep
//     its shifts at fixed word offsets it runs on the normalised modulus
//     q' = q * 2^s whose bit length is the top of the width class,
//     T = 32W - 4 (60, 124 or 252 bits; s = T - bitlen(q)).  With k = 2T:
//     mu = floor(2^(2T)/q'), q1 = floor(x / 2^(T-1)), q3 = floor(q1*mu /
//     2^(T+1)), r = x - q3*q'.  q3 is at most 2 below floor(x/q') (plus 1 for
//     the dropped low columns of q1*mu with W=4 and W=8), so r < 4q' and two
//     conditional subtractions make it canonical.  Multiplying a*2^s by b
//     modulo q' gives 2^s * (a*b mod q), and a right shift by s returns the
//     residue mod q.  A modulus at the top of its class has s = 0 and skips
//     both shifts (a uniform branch).
//
// Everything here is device code; host-side constants (w', mu) are produced by
// the plan code with exact long division.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mw {

typedef uint32_t u32;
typedef uint64_t u64;

template <int W>
struct Res {
  u32 v[W];
};

// Per-modulus constants, passed by value as a kernel argument (uniform).
template <int W>
struct Modulus {
  u32 q[W];
  u32 q2[W];   // 2q
  u32 q4[W];   // 4q
  u32 q8[W];   // 8q
  u32 negq[W]; // 2^(32W) - q
  u32 qn[W];   // Barrett's normalised modulus q' = q * 2^shift, bitlen(q') = 32W - 4
  u32 qn2[W];  // 2q'
  u32 mu[W];   // Barrett mu = floor(2^(2(32W-4)) / q') (32W-3 bits)
  u32 bits;    // b = bitlen(q)
  u32 shift;   // (32W - 4) - b
  u32 est_rcp; // bits of a float just below 1 / (q_top + 1), q_top = q's top word
  u32 est_ok;  // 1: q_top >= 2^16, so canon16 may estimate the quotient from it
};

// Bit length of a normalised Barrett modulus of W words.
template <int W>
constexpr int barrett_bits() { return 32 * W - 4; }

// ---------------------------------------------------------------------------
// word-level primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }
__device__ __forceinline__ u64 pack(u32 lo, u32 hi) { return ((u64)hi << 32) | lo; }

// The three instruction wrappers below are the only CDNA-specific code of the
// arithmetic.  An includer that defines MW_ISA_EMULATED supplies its own
// mad_cc / add_carry / funnel with the same contracts (the CPU emulation test
// does, to run this header's routines on the host).
#ifndef MW_ISA_EMULATED
// acc = a*b + acc (mod 2^64); returns the carry-out lane mask.
__device__ __forceinline__ u64 mad_cc(u32 a, u32 b, u64& acc) {
  u64 cc;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(cc) : "v"(a), "v"(b));
  return cc;
}

// x + carry(cc) where cc is a lane mask produced by a carry-out.
__device__ __forceinline__ u32 add_carry(u32 x, u64 cc) {
  u32 d;
  u64 co;
  asm("v_addc_co_u32 %0, %1, %2, 0, %3" : "=v"(d), "=s"(co) : "v"(x), "s"(cc));
  return d;
}

// funnel shift: bits [s, s+32) of the 64-bit value hi:lo, 0 <= s < 32
__device__ __forceinline__ u32 funnel(u32 hi, u32 lo, u32 s) { return __builtin_amdgcn_alignbit(hi, lo, s); }
#endif

// plain a*b + c, no carry needed (caller guarantees no overflow, or only
// the result modulo 2^64 is used)
__device__ __forceinline__ u64 mad(u32 a, u32 b, u64 c) { return (u64)a * b + c; }

// ---------------------------------------------------------------------------
// multi-word add / sub / compare-select
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ Res<W> add(const Res<W>& a, const Res<W>& b) {
  Res<W> r;
  u32 c = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = __builtin_addc(a.v[i], b.v[i], c, &c);
  return r;
}

template <int W>
__device__ __forceinline__ Res<W> add(const Res<W>& a, const u32 (&b)[W]) {
  Res<W> r;
  u32 c = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = __builtin_addc(a.v[i], b[i], c, &c);
  return r;
}

template <int W>
__device__ __forceinline__ Res<W> sub(const Res<W>& a, const Res<W>& b, u32& borrow) {
  Res<W> r;
  u32 c = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = __builtin_subc(a.v[i], b.v[i], c, &c);
  borrow = c;
  return r;
}

template <int W>
__device__ __forceinline__ Res<W> sub(const Res<W>& a, const u32 (&b)[W], u32& borrow) {
  Res<W> r;
  u32 c = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = __builtin_subc(a.v[i], b[i], c, &c);
  borrow = c;
  return r;
}

// a >= m ? a - m : a   (Eq. saddmod's conditional subtraction)
template <int W>
__device__ __forceinline__ Res<W> csub(const Res<W>& a, const u32 (&m)[W]) {
  u32 borrow;
  Res<W> d = sub(a, m, borrow);
  Res<W> r;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = borrow ? a.v[i] : d.v[i];
  return r;
}

// canonical (a + b) mod q for a, b in [0, q)   (Eq. saddmod)
template <int W>
__device__ __forceinline__ Res<W> addmod(const Res<W>& a, const Res<W>& b, const Modulus<W>& M) {
  return csub(add(a, b), M.q);
}

// canonical (a - b) mod q for a, b in [0, q)   (Eq. ssubmod)
template <int W>
__device__ __forceinline__ Res<W> submod(const Res<W>& a, const Res<W>& b, const Modulus<W>& M) {
  u32 borrow;
  Res<W> d = sub(a, b, borrow);
  Res<W> e = add(d, M.q);
  Res<W> r;
#pragma unroll
  for (int i = 0; i < W; ++i) r.v[i] = borrow ? e.v[i] : d.v[i];
  return r;
}

// ---------------------------------------------------------------------------
// products
// ---------------------------------------------------------------------------

// low W words of a*b
__device__ __forceinline__ Res<4> mul_lo(const Res<4>& a, const u32 (&b)[4]) {
  Res<4> r;
  u64 c0 = (u64)a.v[0] * b[0];
  r.v[0] = lo32(c0);
  u64 c1 = mad(a.v[0], b[1], (u64)hi32(c0));          // < 2^64, no carry
  u64 cc = mad_cc(a.v[1], b[0], c1);
  r.v[1] = lo32(c1);
  u64 c2 = pack(hi32(c1), add_carry(0u, cc));         // carry from column 1
  c2 = mad(a.v[0], b[2], c2);                         // column 2 modulo 2^64:
  c2 = mad(a.v[1], b[1], c2);                         // only its low 64 bits reach
  c2 = mad(a.v[2], b[0], c2);                         // words 2 and 3
  r.v[2] = lo32(c2);
  u64 c3 = (u64)hi32(c2);
  c3 = mad(a.v[0], b[3], c3);                         // column 3: low word only
  c3 = mad(a.v[1], b[2], c3);
  c3 = mad(a.v[2], b[1], c3);
  c3 = mad(a.v[3], b[0], c3);
  r.v[3] = lo32(c3);
  return r;
}

__device__ __forceinline__ Res<2> mul_lo(const Res<2>& a, const u32 (&b)[2]) {
  Res<2> r;
  u64 c0 = (u64)a.v[0] * b[0];
  r.v[0] = lo32(c0);
  u64 c1 = (u64)hi32(c0);
  c1 = mad(a.v[0], b[1], c1);
  c1 = mad(a.v[1], b[0], c1);
  r.v[1] = lo32(c1);
  return r;
}

// low W words of x*w + Q*nq: the Shoup remainder x*w - Q*q modulo 2^(32W)
// when nq = 2^(32W) - q, as one accumulation.
__device__ __forceinline__ Res<4> mul_lo2(const Res<4>& x, const u32 (&w)[4], const Res<4>& Q, const u32 (&nq)[4]) {
  Res<4> r;
  // column 0
  u64 acc = (u64)x.v[0] * w[0];
  u64 cc = mad_cc(Q.v[0], nq[0], acc);
  u32 t = add_carry(0u, cc);
  r.v[0] = lo32(acc);
  // column 1: carry-in {hi, t} < 2^33 so the first product cannot overflow
  acc = pack(hi32(acc), t);
  acc = mad(x.v[0], w[1], acc);
  cc = mad_cc(x.v[1], w[0], acc);
  t = add_carry(0u, cc);
  cc = mad_cc(Q.v[0], nq[1], acc);
  t = add_carry(t, cc);
  cc = mad_cc(Q.v[1], nq[0], acc);
  t = add_carry(t, cc);
  r.v[1] = lo32(acc);
  // column 2 modulo 2^64 (only its low 64 bits reach words 2 and 3)
  acc = pack(hi32(acc), t);
  acc = mad(x.v[0], w[2], acc);
  acc = mad(x.v[1], w[1], acc);
  acc = mad(x.v[2], w[0], acc);
  acc = mad(Q.v[0], nq[2], acc);
  acc = mad(Q.v[1], nq[1], acc);
  acc = mad(Q.v[2], nq[0], acc);
  r.v[2] = lo32(acc);
  // column 3: low word only
  u32 c3 = hi32(acc);
  c3 += x.v[0] * w[3] + x.v[1] * w[2] + x.v[2] * w[1] + x.v[3] * w[0];
  c3 += Q.v[0] * nq[3] + Q.v[1] * nq[2] + Q.v[2] * nq[1] + Q.v[3] * nq[0];
  r.v[3] = c3;
  return r;
}

__device__ __forceinline__ Res<2> mul_lo2(const Res<2>& x, const u32 (&w)[2], const Res<2>& Q, const u32 (&nq)[2]) {
  Res<2> r;
  u64 acc = (u64)x.v[0] * w[0];
  acc = mad(Q.v[0], nq[0], acc);        // column 0 modulo 2^64: only its high word is used below
  r.v[0] = lo32(acc);
  u32 c1 = hi32(acc);
  c1 += x.v[0] * w[1] + x.v[1] * w[0] + Q.v[0] * nq[1] + Q.v[1] * nq[0];
  r.v[1] = c1;
  return r;
}

// Shoup quotient estimate: floor(sum over columns >= W-1 of x*ws / 2^(32W)).
// Under-estimates floor(x*ws / 2^(32W)) by at most 4 (W=4) / 1 (W=2).
__device__ __forceinline__ Res<4> mul_hi_est(const Res<4>& x, const u32 (&ws)[4]) {
  Res<4> Q;
  // column 3
  u64 acc = (u64)x.v[0] * ws[3];
  u64 cc = mad_cc(x.v[1], ws[2], acc);
  u32 t = add_carry(0u, cc);
  cc = mad_cc(x.v[2], ws[1], acc);
  t = add_carry(t, cc);
  cc = mad_cc(x.v[3], ws[0], acc);
  t = add_carry(t, cc);
  // column 4
  acc = pack(hi32(acc), t);
  cc = mad_cc(x.v[1], ws[3], acc);
  t = add_carry(0u, cc);
  cc = mad_cc(x.v[2], ws[2], acc);
  t = add_carry(t, cc);
  cc = mad_cc(x.v[3], ws[1], acc);
  t = add_carry(t, cc);
  Q.v[0] = lo32(acc);
  // column 5
  acc = pack(hi32(acc), t);
  cc = mad_cc(x.v[2], ws[3], acc);
  t = add_carry(0u, cc);
  cc = mad_cc(x.v[3], ws[2], acc);
  t = add_carry(t, cc);
  Q.v[1] = lo32(acc);
  // column 6 (+7): the estimate is below 2^128, so no carry leaves it
  acc = pack(hi32(acc), t);
  acc = mad(x.v[3], ws[3], acc);
  Q.v[2] = lo32(acc);
  Q.v[3] = hi32(acc);
  return Q;
}

__device__ __forceinline__ Res<2> mul_hi_est(const Res<2>& x, const u32 (&ws)[2]) {
  Res<2> Q;
  u64 acc = (u64)x.v[0] * ws[1];                      // column 1
  u64 cc = mad_cc(x.v[1], ws[0], acc);
  u32 t = add_carry(0u, cc);
  acc = pack(hi32(acc), t);                           // column 2 (+3)
  acc = mad(x.v[1], ws[1], acc);
  Q.v[0] = lo32(acc);
  Q.v[1] = hi32(acc);
  return Q;
}

// Full 2W-word product a*b.
__device__ __forceinline__ void mul_full(const Res<4>& a, const Res<4>& b, u32 (&r)[8]) {
  u64 acc = (u64)a.v[0] * b.v[0];
  r[0] = lo32(acc);
  // column 1
  acc = (u64)hi32(acc);
  acc = mad(a.v[0], b.v[1], acc);
  u64 cc = mad_cc(a.v[1], b.v[0], acc);
  u32 t = add_carry(0u, cc);
  r[1] = lo32(acc);
  // column 2
  acc = pack(hi32(acc), t);
  cc = mad_cc(a.v[0], b.v[2], acc);
  t = add_carry(0u, cc);
  cc = mad_cc(a.v[1], b.v[1], acc);
  t = add_carry(t, cc);
  cc = mad_cc(a.v[2], b.v[0], acc);
  t = add_carry(t, cc);
  r[2] = lo32(acc);
  // column 3
  acc = pack(hi32(acc), t);
  cc = mad_cc(a.v[0], b.v[3], acc);
  t = add_carry(0u, cc);
  cc = mad_cc(a.v[1], b.v[2], acc);
  t = add_carry(t, cc);
  cc = mad_cc(a.v[2], b.v[1], acc);
  t = add_carry(t, cc);
  cc = mad_cc(a.v[3], b.v[0], acc);
  t = add_carry(t, cc);
  r[3] = lo32(acc);
  // column 4
  acc = pack(hi32(acc), t);
  cc = mad_cc(a.v[1], b.v[3], acc);
  t = add_carry(0u, cc);
  cc = mad_cc(a.v[2], b.v[2], acc);
  t = add_carry(t, cc);
  cc = mad_cc(a.v[3], b.v[1], acc);
  t = add_carry(t, cc);
  r[4] = lo32(acc);
  // column 5
  acc = pack(hi32(acc), t);
  cc = mad_cc(a.v[2], b.v[3], acc);
  t = add_carry(0u, cc);
  cc = mad_cc(a.v[3], b.v[2], acc);
  t = add_carry(t, cc);
  r[5] = lo32(acc);
  // column 6 (+7)
  acc = pack(hi32(acc), t);
  acc = mad(a.v[3], b.v[3], acc);
  r[6] = lo32(acc);
  r[7] = hi32(acc);
}

__device__ __forceinline__ void mul_full(const Res<2>& a, const Res<2>& b, u32 (&r)[4]) {
  u64 acc = (u64)a.v[0] * b.v[0];
  r[0] = lo32(acc);
  acc = (u64)hi32(acc);
  acc = mad(a.v[0], b.v[1], acc);
  u64 cc = mad_cc(a.v[1], b.v[0], acc);
  u32 t = add_carry(0u, cc);
  r[1] = lo32(acc);
  acc = pack(hi32(acc), t);
  acc = mad(a.v[1], b.v[1], acc);
  r[2] = lo32(acc);
  r[3] = hi32(acc);
}

// ---------------------------------------------------------------------------
// Generic W-word products (used for W = 8, four 64-bit limbs).  Product
// scanning: column c of a*b is the sum of a_i * b_(c-i); a 64-bit accumulator
// takes the products of a column with their carry-outs counted in t, and the
// next column starts from {hi(acc), t}.  All loop bounds are compile-time
// constants, so everything unrolls to straight-line code.
// ---------------------------------------------------------------------------

// Columns C0..2W-2 of a*b accumulated from column C0 upward (the columns
// below C0 are not added): out[c - C0] = word c for C0 <= c <= 2W-1.  The
// truncated sum is below 2^(64W), so nothing carries out of the top word.
template <int W, int C0>
__device__ __forceinline__ void mul_cols(const u32 (&a)[W], const u32 (&b)[W], u32 (&out)[2 * W - C0]) {
  u64 acc = 0;
  u32 t = 0;
#pragma unroll
  for (int c = C0; c <= 2 * W - 2; ++c) {
    const int i0 = c > W - 1 ? c - (W - 1) : 0;
    const int i1 = c < W - 1 ? c : W - 1;
    if (c > C0) acc = pack(hi32(acc), t);
    t = 0;
#pragma unroll
    for (int i = i0; i <= i1; ++i) {
      if (c == C0 && i == i0) {
        acc = (u64)a[i] * b[c - i];
      } else if (c == 2 * W - 2) {
        acc = mad(a[i], b[c - i], acc);     // top column: the sum fits
      } else {
        const u64 cc = mad_cc(a[i], b[c - i], acc);
        t = add_carry(t, cc);
      }
    }
    out[c - C0] = lo32(acc);
  }
  out[2 * W - 1 - C0] = hi32(acc);
}

// Full 2W-word product by one level of Karatsuba (Eq. mulk) on W/2-word
// halves a = a1*B + a0, b = b1*B + b0, B = 2^(16W):
//   a*b = z2*B^2 + z1*B + z0, z0 = a0*b0, z2 = a1*b1,
//   z1 = (a0 + a1)(b0 + b1) - z0 - z2 = a0*b1 + a1*b0 < 2*B^2.
// The half sums carry one bit each (ca, cb), so the middle product is
// m + (ca*sb + cb*sa)*B + ca*cb*B^2 with m = sa*sb; three half products of
// (W/2)^2 word products replace the W^2 of the schoolbook product, at the
// price of the half sums, the carry corrections and the two subtractions.
template <int W>
__device__ __forceinline__ void mul_full_kara(const u32 (&a)[W], const u32 (&b)[W], u32 (&r)[2 * W]) {
  constexpr int H = W / 2;
  u32 a0[H], a1[H], b0[H], b1[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    a0[i] = a[i];
    a1[i] = a[H + i];
    b0[i] = b[i];
    b1[i] = b[H + i];
  }
  u32 z0[2 * H], z2[2 * H], m[2 * H];
  mul_cols<H, 0>(a0, b0, z0);
  mul_cols<H, 0>(a1, b1, z2);
  u32 sa[H], sb[H], ca = 0, cb = 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    sa[i] = __builtin_addc(a0[i], a1[i], ca, &ca);
    sb[i] = __builtin_addc(b0[i], b1[i], cb, &cb);
  }
  mul_cols<H, 0>(sa, sb, m);
  // middle product, 2H + 1 words: m + (ca ? sb : 0)*B + (cb ? sa : 0)*B + ca*cb*B^2
  const u32 ma = 0u - ca, mb = 0u - cb;
  u32 top = ca & cb, c1 = 0, c2 = 0;
#pragma unroll
  for (int i = 0; i < H; ++i) m[H + i] = __builtin_addc(m[H + i], sb[i] & ma, c1, &c1);
#pragma unroll
  for (int i = 0; i < H; ++i) m[H + i] = __builtin_addc(m[H + i], sa[i] & mb, c2, &c2);
  top += c1 + c2;
  // z1 = middle - z0 - z2 (non-negative, below 2^(64H+1))
  u32 d1 = 0, d2 = 0;
#pragma unroll
  for (int i = 0; i < 2 * H; ++i) m[i] = __builtin_subc(m[i], z0[i], d1, &d1);
  top -= d1;
#pragma unroll
  for (int i = 0; i < 2 * H; ++i) m[i] = __builtin_subc(m[i], z2[i], d2, &d2);
  top -= d2;
  // r = z2*B^2 + z0, plus z1 at word H (the sum is below 2^(64W): no carry out)
#pragma unroll
  for (int i = 0; i < 2 * H; ++i) {
    r[i] = z0[i];
    r[2 * H + i] = z2[i];
  }
  u32 c = 0;
#pragma unroll
  for (int i = 0; i < 2 * H; ++i) r[H + i] = __builtin_addc(r[H + i], m[i], c, &c);
  r[3 * H] = __builtin_addc(r[3 * H], top, c, &c);
#pragma unroll
  for (int i = 3 * H + 1; i < 2 * W; ++i) r[i] = __builtin_addc(r[i], 0u, c, &c);
}

// Low W words of a*b (+ c*d when TWO) (columns 0..W-1; column W-2 is only
// needed modulo 2^64 and column W-1 modulo 2^32).
template <int W, bool TWO>
__device__ __forceinline__ void mul_lo_sum(const u32 (&a)[W], const u32 (&b)[W], const u32 (&c)[W],
                                           const u32 (&d)[W], u32 (&out)[W]) {
  u64 acc = 0;
  u32 t = 0;
#pragma unroll
  for (int col = 0; col <= W - 3; ++col) {
    if (col > 0) acc = pack(hi32(acc), t);
    t = 0;
#pragma unroll
    for (int i = 0; i <= col; ++i) {
      if (col == 0 && i == 0) {
        acc = (u64)a[0] * b[0];
      } else {
        const u64 cc = mad_cc(a[i], b[col - i], acc);
        t = add_carry(t, cc);
      }
    }
    if constexpr (TWO) {
#pragma unroll
      for (int i = 0; i <= col; ++i) {
        const u64 cc = mad_cc(c[i], d[col - i], acc);
        t = add_carry(t, cc);
      }
    }
    out[col] = lo32(acc);
  }
  acc = pack(hi32(acc), t);
#pragma unroll
  for (int i = 0; i <= W - 2; ++i) {
    acc = mad(a[i], b[W - 2 - i], acc);
    if constexpr (TWO) acc = mad(c[i], d[W - 2 - i], acc);
  }
  out[W - 2] = lo32(acc);
  u32 top = hi32(acc);
#pragma unroll
  for (int i = 0; i <= W - 1; ++i) {
    top += a[i] * b[W - 1 - i];
    if constexpr (TWO) top += c[i] * d[W - 1 - i];
  }
  out[W - 1] = top;
}

// Shoup quotient estimate for W = 8: columns >= W-2 of x*ws.  The dropped
// columns sum to less than 6 * 2^224 * (1 + 2^-32), so the estimate is at
// most 1 below floor(x*ws / 2^256) and x*w - Q*q lies in [0, 3q).
__device__ __forceinline__ Res<8> mul_hi_est(const Res<8>& x, const u32 (&ws)[8]) {
  u32 cols[10];
  mul_cols<8, 6>(x.v, ws, cols);
  Res<8> Q;
#pragma unroll
  for (int k = 0; k < 8; ++k) Q.v[k] = cols[k + 2];
  return Q;
}

__device__ __forceinline__ Res<8> mul_lo2(const Res<8>& x, const u32 (&w)[8], const Res<8>& Q, const u32 (&nq)[8]) {
  Res<8> r;
  mul_lo_sum<8, true>(x.v, w, Q.v, nq, r.v);
  return r;
}

__device__ __forceinline__ Res<8> mul_lo(const Res<8>& a, const u32 (&b)[8]) {
  Res<8> r;
  mul_lo_sum<8, false>(a.v, b, b, b, r.v);
  return r;
}

// ---------------------------------------------------------------------------
// modular multiplication
// ---------------------------------------------------------------------------

// Shoup: x*w mod q up to a multiple of q, result in [0, 6q), for x < 2^(32W),
// w < q, ws = floor(w * 2^(32W) / q).
template <int W>
__device__ __forceinline__ Res<W> shoup_mul(const Res<W>& x, const u32 (&w)[W], const u32 (&ws)[W],
                                            const Modulus<W>& M) {
  Res<W> Q = mul_hi_est(x, ws);
  return mul_lo2(x, w, Q, M.negq);
}

// Word moves of the uniform shifts: by K, 2K, 4K, ... words where the
// corresponding bit of ws is set, as selects (every index a compile-time
// constant, so the residue stays in registers).
template <int W, int K>
__device__ __forceinline__ void words_up(Res<W>& t, u32 ws) {
  if constexpr (K < W) {
    const bool on = (ws & (u32)K) != 0;
#pragma unroll
    for (int i = W - 1; i >= 0; --i) t.v[i] = on ? (i >= K ? t.v[i - K] : 0u) : t.v[i];
    words_up<W, 2 * K>(t, ws);
  }
}

template <int W, int K>
__device__ __forceinline__ void words_down(Res<W>& t, u32 ws) {
  if constexpr (K < W) {
    const bool on = (ws & (u32)K) != 0;
#pragma unroll
    for (int i = 0; i < W; ++i) t.v[i] = on ? (i + K < W ? t.v[i + K] : 0u) : t.v[i];
    words_down<W, 2 * K>(t, ws);
  }
}

// a * 2^s for a uniform 0 < s < 32W whose result fits in W words: a word
// shift by s / 32 in log2(W) uniform steps, then a bit shift by s % 32.
template <int W>
__device__ __forceinline__ Res<W> shl_uniform(const Res<W>& a, u32 s) {
  Res<W> t = a;
  words_up<W, 1>(t, s >> 5);
  const u32 bs = s & 31;
  Res<W> r;
#pragma unroll
  for (int i = W - 1; i > 0; --i) r.v[i] = bs ? funnel(t.v[i], t.v[i - 1], 32u - bs) : t.v[i];
  r.v[0] = t.v[0] << bs;
  return r;
}

// a / 2^s for a uniform 0 < s < 32W (exact here: a is a multiple of 2^s).
template <int W>
__device__ __forceinline__ Res<W> shr_uniform(const Res<W>& a, u32 s) {
  Res<W> t = a;
  words_down<W, 1>(t, s >> 5);
  const u32 bs = s & 31;
  Res<W> r;
#pragma unroll
  for (int i = 0; i < W - 1; ++i) r.v[i] = funnel(t.v[i + 1], t.v[i], bs);
  r.v[W - 1] = t.v[W - 1] >> bs;
  return r;
}

// Barrett core on the normalised modulus (T = 124 bits): canonical x mod q'
// for x = a*b < 2^248.  The shifts by T - 1 = 123 and T + 1 = 125 bits start
// in word 3 at bit offsets 27 and 29.
template <bool KARA = false>
__device__ __forceinline__ Res<4> barrett_core(const Res<4>& a, const Res<4>& b, const Modulus<4>& M) {
  u32 x[8];
  if constexpr (KARA) mul_full_kara<4>(a.v, b.v, x);
  else mul_full(a, b, x);
  constexpr u32 s1 = (barrett_bits<4>() - 1) & 31;
  Res<4> q1;
  q1.v[0] = funnel(x[4], x[3], s1);
  q1.v[1] = funnel(x[5], x[4], s1);
  q1.v[2] = funnel(x[6], x[5], s1);
  q1.v[3] = funnel(x[7], x[6], s1);
  // q2 = q1 * mu, columns >= 2 (dropped part < 2^98 < 2^(T+1))
  u32 q2[8];
  {
    const u32* m = M.mu;
    u64 acc = (u64)q1.v[0] * m[2];
    u64 cc = mad_cc(q1.v[1], m[1], acc);
    u32 t = add_carry(0u, cc);
    cc = mad_cc(q1.v[2], m[0], acc);
    t = add_carry(t, cc);
    q2[2] = lo32(acc);
    acc = pack(hi32(acc), t);
    cc = mad_cc(q1.v[0], m[3], acc);
    t = add_carry(0u, cc);
    cc = mad_cc(q1.v[1], m[2], acc);
    t = add_carry(t, cc);
    cc = mad_cc(q1.v[2], m[1], acc);
    t = add_carry(t, cc);
    cc = mad_cc(q1.v[3], m[0], acc);
    t = add_carry(t, cc);
    q2[3] = lo32(acc);
    acc = pack(hi32(acc), t);
    cc = mad_cc(q1.v[1], m[3], acc);
    t = add_carry(0u, cc);
    cc = mad_cc(q1.v[2], m[2], acc);
    t = add_carry(t, cc);
    cc = mad_cc(q1.v[3], m[1], acc);
    t = add_carry(t, cc);
    q2[4] = lo32(acc);
    acc = pack(hi32(acc), t);
    cc = mad_cc(q1.v[2], m[3], acc);
    t = add_carry(0u, cc);
    cc = mad_cc(q1.v[3], m[2], acc);
    t = add_carry(t, cc);
    q2[5] = lo32(acc);
    acc = pack(hi32(acc), t);
    acc = mad(q1.v[3], m[3], acc);
    q2[6] = lo32(acc);
    q2[7] = hi32(acc);
  }
  constexpr u32 s3 = (barrett_bits<4>() + 1) & 31;
  Res<4> q3;
  q3.v[0] = funnel(q2[4], q2[3], s3);
  q3.v[1] = funnel(q2[5], q2[4], s3);
  q3.v[2] = funnel(q2[6], q2[5], s3);
  q3.v[3] = funnel(q2[7], q2[6], s3);
  // r = x - q3*q'  (mod 2^128; the true value is in [0, 4q'))
  Res<4> xl;
  xl.v[0] = x[0]; xl.v[1] = x[1]; xl.v[2] = x[2]; xl.v[3] = x[3];
  Res<4> qq = mul_lo(q3, M.qn);
  u32 bo;
  Res<4> r = sub(xl, qq, bo);
  r = csub(r, M.qn2);
  return csub(r, M.qn);
}

// T = 60 bits: the shifts by 59 and 61 bits start in word 1.
template <bool KARA = false>
__device__ __forceinline__ Res<2> barrett_core(const Res<2>& a, const Res<2>& b, const Modulus<2>& M) {
  u32 x[4];
  if constexpr (KARA) mul_full_kara<2>(a.v, b.v, x);
  else mul_full(a, b, x);
  constexpr u32 s1 = (barrett_bits<2>() - 1) & 31;
  Res<2> q1;
  q1.v[0] = funnel(x[2], x[1], s1);
  q1.v[1] = funnel(x[3], x[2], s1);
  Res<2> mu;
  mu.v[0] = M.mu[0];
  mu.v[1] = M.mu[1];
  u32 q2[4];
  mul_full(q1, mu, q2);
  constexpr u32 s3 = (barrett_bits<2>() + 1) & 31;
  Res<2> q3;
  q3.v[0] = funnel(q2[2], q2[1], s3);
  q3.v[1] = funnel(q2[3], q2[2], s3);
  Res<2> xl;
  xl.v[0] = x[0]; xl.v[1] = x[1];
  Res<2> qq = mul_lo(q3, M.qn);
  u32 bo;
  Res<2> r = sub(xl, qq, bo);
  r = csub(r, M.qn2);
  return csub(r, M.qn);
}

// T = 252 bits: the shifts by 251 and 253 bits start in word 7; q1*mu drops
// columns 0..4 (less than 5 * 2^192 * (1 + 2^-32) < 2^(T+1)), so q3 is at
// most 3 below floor(x/q') and r < 4q'.
template <bool KARA = false>
__device__ __forceinline__ Res<8> barrett_core(const Res<8>& a, const Res<8>& b, const Modulus<8>& M) {
  u32 x[16];
  if constexpr (KARA) mul_full_kara<8>(a.v, b.v, x);
  else mul_cols<8, 0>(a.v, b.v, x);
  constexpr u32 s1 = (barrett_bits<8>() - 1) & 31;
  Res<8> q1;
#pragma unroll
  for (int k = 0; k < 8; ++k) q1.v[k] = funnel(x[8 + k], x[7 + k], s1);
  u32 q2[11];   // words 5..15 of the truncated q1*mu
  mul_cols<8, 5>(q1.v, M.mu, q2);
  constexpr u32 s3 = (barrett_bits<8>() + 1) & 31;
  Res<8> q3;
#pragma unroll
  for (int k = 0; k < 8; ++k) q3.v[k] = funnel(q2[3 + k], q2[2 + k], s3);   // words 8+k : 7+k
  Res<8> xl;
#pragma unroll
  for (int k = 0; k < 8; ++k) xl.v[k] = x[k];
  Res<8> qq = mul_lo(q3, M.qn);
  u32 bo;
  Res<8> r = sub(xl, qq, bo);
  r = csub(r, M.qn2);
  return csub(r, M.qn);
}

// Barrett: canonical a*b mod q for a, b in [0, q), any odd q of the width
// class.  a*2^s < q' and b < q <= q', so x = a*2^s*b < 2^(2T).  NORM (known
// at compile time) selects the scaled form (M.shift > 0) or the plain one
// (M.shift == 0); barrett_mul decides at run time with a uniform branch.
// KARA: the full product a*b by one level of Karatsuba instead of the
// schoolbook columns (the other two products of the reduction are truncated,
// and stay schoolbook).
template <int W, bool NORM, bool KARA = false>
__device__ __forceinline__ Res<W> barrett_mul_t(const Res<W>& a, const Res<W>& b, const Modulus<W>& M) {
  if constexpr (NORM) return shr_uniform(barrett_core<KARA>(shl_uniform(a, M.shift), b, M), M.shift);
  else return barrett_core<KARA>(a, b, M);
}

template <int W>
__device__ __forceinline__ Res<W> barrett_mul(const Res<W>& a, const Res<W>& b, const Modulus<W>& M) {
  if (M.shift == 0) return barrett_mul_t<W, false>(a, b, M);
  return barrett_mul_t<W, true>(a, b, M);
}

// ---------------------------------------------------------------------------
// loads / stores of one residue (W words, 16-byte or 8-byte aligned)
// ---------------------------------------------------------------------------
__device__ __forceinline__ Res<4> load_res(const void* p) {
  uint4 v = *reinterpret_cast<const uint4*>(p);
  Res<4> r;
  r.v[0] = v.x; r.v[1] = v.y; r.v[2] = v.z; r.v[3] = v.w;
  return r;
}
__device__ __forceinline__ void store_res(void* p, const Res<4>& r) {
  *reinterpret_cast<uint4*>(p) = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
}
__device__ __forceinline__ Res<2> load_res2(const void* p) {
  uint2 v = *reinterpret_cast<const uint2*>(p);
  Res<2> r;
  r.v[0] = v.x; r.v[1] = v.y;
  return r;
}
__device__ __forceinline__ void store_res2(void* p, const Res<2>& r) {
  *reinterpret_cast<uint2*>(p) = make_uint2(r.v[0], r.v[1]);
}

template <int W> struct ResIO;
template <> struct ResIO<4> {
  __device__ static __forceinline__ Res<4> load(const void* p) { return load_res(p); }
  __device__ static __forceinline__ void store(void* p, const Res<4>& r) { store_res(p, r); }
};
template <> struct ResIO<8> {
  __device__ static __forceinline__ Res<8> load(const void* p) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    const uint4 lo = q[0], hi = q[1];
    Res<8> r;
    r.v[0] = lo.x; r.v[1] = lo.y; r.v[2] = lo.z; r.v[3] = lo.w;
    r.v[4] = hi.x; r.v[5] = hi.y; r.v[6] = hi.z; r.v[7] = hi.w;
    return r;
  }
  __device__ static __forceinline__ void store(void* p, const Res<8>& r) {
    uint4* q = reinterpret_cast<uint4*>(p);
    q[0] = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
    q[1] = make_uint4(r.v[4], r.v[5], r.v[6], r.v[7]);
  }
};
template <> struct ResIO<2> {
  __device__ static __forceinline__ Res<2> load(const void* p) { return load_res2(p); }
  __device__ static __forceinline__ void store(void* p, const Res<2>& r) { store_res2(p, r); }
};

}  // namespace mw
