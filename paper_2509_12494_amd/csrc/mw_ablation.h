// Arithmetic variants of the two-word (124-bit) butterfly for the GPU analog of
// the paper's MQX ablation (Evaluation, sensitivity to the MQX components;
// Table tab:mqx lists them: a widening multiply, add/sub with carry, a
// multiply-high substitute, predicated carries).  On CDNA4 every component
// exists natively; each variant removes one from the native butterfly of
// mw_butterfly.h while computing the same values:
//
//   IsaMulHi    no widening multiply-add: a 32x32 product is v_mul_lo_u32 and
//               v_mul_hi_u32, added into the column with a carry-chain add;
//   IsaCmpCarry no carry flags consumed: the carry of a column add, of a
//               multi-word add or subtract is recovered by an unsigned compare
//               of the result with an operand and a select, instead of the
//               carry-out / carry-in of v_mad_u64_u32, v_addc_co_u32 and
//               v_subb_co_u32 (the widening multiply stays);
//   IsaPlain    both removed.
//
// The column structure, lazy ranges and reduction bounds are those of
// mw_arith.h / mw_butterfly.h; only the instructions that realise them change.
#pragma once
#include "mw_butterfly.h"

namespace mw {

// ---------------------------------------------------------------------------
// primitives per variant: prod(a, b) = a*b as 64 bits; mad_cc adds a*b into a
// 64-bit accumulator and returns the carry out (0 or 1); add_c / sub_b are one
// word of a carry / borrow chain (carries as 0/1 values).
// ---------------------------------------------------------------------------
struct IsaMulHiBase {
  static __device__ __forceinline__ u64 prod(u32 a, u32 b) {
    u32 lo, hi;
    asm("v_mul_lo_u32 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
    asm("v_mul_hi_u32 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
    return pack(lo, hi);
  }
  template <class Carry>
  static __device__ __forceinline__ u64 mad(u32 a, u32 b, u64 c) { return Carry::add64(prod(a, b), c); }
};

struct IsaWideBase {
  static __device__ __forceinline__ u64 prod(u32 a, u32 b) { return (u64)a * b; }
  // the widening multiply-add itself (its carry-out unused)
  template <class Carry>
  static __device__ __forceinline__ u64 mad(u32 a, u32 b, u64 c) { return (u64)a * b + c; }
};

// carries from the hardware carry chain
struct CarryFlags {
  static __device__ __forceinline__ u32 add_c(u32 a, u32 b, u32 cin, u32& cout) {
    return __builtin_addc(a, b, cin, &cout);
  }
  static __device__ __forceinline__ u32 sub_b(u32 a, u32 b, u32 bin, u32& bout) {
    return __builtin_subc(a, b, bin, &bout);
  }
  // a + b mod 2^64
  static __device__ __forceinline__ u64 add64(u64 a, u64 b) { return a + b; }
  // acc += p (64-bit) with the carry out as 0/1
  static __device__ __forceinline__ u32 add64_c(u64& acc, u64 p) {
    u32 c0, c1;
    const u32 lo = __builtin_addc((u32)acc, (u32)p, 0u, &c0);
    const u32 hi = __builtin_addc((u32)(acc >> 32), (u32)(p >> 32), c0, &c1);
    acc = pack(lo, hi);
    return c1;
  }
};

// carries recovered by compare and select.  The 32-bit adds and subtracts are
// single-instruction asm (no carry-out): written in C, the compiler would
// recognise "s < a" after "s = a + b" as the add's overflow and turn the pair
// back into a carry-producing add.
struct CarryCompare {
  static __device__ __forceinline__ u32 add32(u32 a, u32 b) {
    u32 d;
    asm("v_add_u32 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
    return d;
  }
  static __device__ __forceinline__ u32 sub32(u32 a, u32 b) {
    u32 d;
    asm("v_sub_u32 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
    return d;
  }
  static __device__ __forceinline__ u32 add_c(u32 a, u32 b, u32 cin, u32& cout) {
    const u32 s = add32(a, b);
    const u32 r = add32(s, cin);
    cout = (s < a ? 1u : 0u) | (r < s ? 1u : 0u);
    return r;
  }
  static __device__ __forceinline__ u32 sub_b(u32 a, u32 b, u32 bin, u32& bout) {
    const u32 d = sub32(a, b);
    const u32 r = sub32(d, bin);
    bout = (a < b ? 1u : 0u) | (d < bin ? 1u : 0u);
    return r;
  }
  // a + b mod 2^64 by the 64-bit shift-add, which has no carry-out
  static __device__ __forceinline__ u64 add64(u64 a, u64 b) {
    u64 d;
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(d) : "v"(a), "v"(b));
    return d;
  }
  static __device__ __forceinline__ u32 add64_c(u64& acc, u64 p) {
    const u64 s = add64(acc, p);
    const u32 c = s < p ? 1u : 0u;
    acc = s;
    return c;
  }
};

template <class Mul, class Carry>
struct IsaVariant {
  static __device__ __forceinline__ u64 prod(u32 a, u32 b) { return Mul::prod(a, b); }
  static __device__ __forceinline__ u32 mad_cc(u32 a, u32 b, u64& acc) { return Carry::add64_c(acc, Mul::prod(a, b)); }
  // a*b + c where the sum cannot overflow 64 bits (or only its low 64 bits are used)
  static __device__ __forceinline__ u64 mad(u32 a, u32 b, u64 c) { return Mul::template mad<Carry>(a, b, c); }
  static __device__ __forceinline__ u32 add_c(u32 a, u32 b, u32 cin, u32& cout) { return Carry::add_c(a, b, cin, cout); }
  static __device__ __forceinline__ u32 sub_b(u32 a, u32 b, u32 bin, u32& bout) { return Carry::sub_b(a, b, bin, bout); }
};

using IsaMulHi = IsaVariant<IsaMulHiBase, CarryFlags>;
using IsaCmpCarry = IsaVariant<IsaWideBase, CarryCompare>;
using IsaPlain = IsaVariant<IsaMulHiBase, CarryCompare>;

// ---------------------------------------------------------------------------
// two-word residue arithmetic on a variant (the same columns as mw_arith.h)
// ---------------------------------------------------------------------------
template <class I>
struct Arith4 {
  static __device__ __forceinline__ Res<4> add(const Res<4>& a, const u32 (&b)[4]) {
    Res<4> r;
    u32 c = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.v[i] = I::add_c(a.v[i], b[i], c, c);
    return r;
  }
  static __device__ __forceinline__ Res<4> add(const Res<4>& a, const Res<4>& b) { return add(a, b.v); }
  static __device__ __forceinline__ Res<4> sub(const Res<4>& a, const u32 (&b)[4], u32& borrow) {
    Res<4> r;
    u32 c = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.v[i] = I::sub_b(a.v[i], b[i], c, c);
    borrow = c;
    return r;
  }
  static __device__ __forceinline__ Res<4> sub(const Res<4>& a, const Res<4>& b, u32& borrow) {
    return sub(a, b.v, borrow);
  }
  static __device__ __forceinline__ Res<4> csub(const Res<4>& a, const u32 (&m)[4]) {
    u32 borrow;
    const Res<4> d = sub(a, m, borrow);
    Res<4> r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.v[i] = borrow ? a.v[i] : d.v[i];
    return r;
  }

  // Shoup quotient estimate: columns >= 3 of x * ws (at most 4 below the
  // exact quotient, as mul_hi_est of mw_arith.h).
  static __device__ __forceinline__ Res<4> mul_hi_est(const Res<4>& x, const u32 (&ws)[4]) {
    Res<4> Q;
    u64 acc = I::prod(x.v[0], ws[3]);
    u32 t = I::mad_cc(x.v[1], ws[2], acc);
    t += I::mad_cc(x.v[2], ws[1], acc);
    t += I::mad_cc(x.v[3], ws[0], acc);
    acc = pack(hi32(acc), t);                          // column 4
    t = I::mad_cc(x.v[1], ws[3], acc);
    t += I::mad_cc(x.v[2], ws[2], acc);
    t += I::mad_cc(x.v[3], ws[1], acc);
    Q.v[0] = lo32(acc);
    acc = pack(hi32(acc), t);                          // column 5
    t = I::mad_cc(x.v[2], ws[3], acc);
    t += I::mad_cc(x.v[3], ws[2], acc);
    Q.v[1] = lo32(acc);
    acc = pack(hi32(acc), t);                          // column 6 (+7)
    acc = I::mad(x.v[3], ws[3], acc);
    Q.v[2] = lo32(acc);
    Q.v[3] = hi32(acc);
    return Q;
  }

  // low 4 words of x*w + Q*nq (the Shoup remainder modulo 2^128)
  static __device__ __forceinline__ Res<4> mul_lo2(const Res<4>& x, const u32 (&w)[4], const Res<4>& Q,
                                                   const u32 (&nq)[4]) {
    Res<4> r;
    u64 acc = I::prod(x.v[0], w[0]);
    u32 t = I::mad_cc(Q.v[0], nq[0], acc);
    r.v[0] = lo32(acc);
    acc = pack(hi32(acc), t);                          // column 1 (carry-in < 2^33)
    acc = I::mad(x.v[0], w[1], acc);
    t = I::mad_cc(x.v[1], w[0], acc);
    t += I::mad_cc(Q.v[0], nq[1], acc);
    t += I::mad_cc(Q.v[1], nq[0], acc);
    r.v[1] = lo32(acc);
    acc = pack(hi32(acc), t);                          // column 2 modulo 2^64
    acc = I::mad(x.v[0], w[2], acc);
    acc = I::mad(x.v[1], w[1], acc);
    acc = I::mad(x.v[2], w[0], acc);
    acc = I::mad(Q.v[0], nq[2], acc);
    acc = I::mad(Q.v[1], nq[1], acc);
    acc = I::mad(Q.v[2], nq[0], acc);
    r.v[2] = lo32(acc);
    u32 c3 = hi32(acc);                                // column 3: low word only
    c3 += x.v[0] * w[3] + x.v[1] * w[2] + x.v[2] * w[1] + x.v[3] * w[0];
    c3 += Q.v[0] * nq[3] + Q.v[1] * nq[2] + Q.v[2] * nq[1] + Q.v[3] * nq[0];
    r.v[3] = c3;
    return r;
  }

  static __device__ __forceinline__ Res<4> shoup_mul(const Res<4>& x, const u32 (&w)[4], const u32 (&ws)[4],
                                                     const Modulus<4>& M) {
    return mul_lo2(x, w, mul_hi_est(x, ws), M.negq);
  }
};

// The butterflies of mw_butterfly.h on a variant.
template <class I>
struct BflyVariant {
  using A = Arith4<I>;
  template <int W>
  static __device__ __forceinline__ void ct(Res<W>& X, Res<W>& Y, const Tw<W>& t, const Modulus<W>& M) {
    static_assert(W == 4, "arithmetic variants are two-word only");
    const Res<4> T = A::shoup_mul(Y, t.w, t.ws, M);
    const Res<4> Xr = A::csub(X, M.q8);
    X = A::add(Xr, T);
    const Res<4> D = A::add(Xr, M.q8);
    u32 b;
    Y = A::sub(D, T, b);
  }
  template <int W>
  static __device__ __forceinline__ void gs(Res<W>& X, Res<W>& Y, const Tw<W>& t, const Modulus<W>& M) {
    const Res<4> S = A::csub(A::add(X, Y), M.q8);
    Res<4> D = A::add(X, M.q8);
    u32 b;
    D = A::sub(D, Y, b);
    Y = A::shoup_mul(D, t.w, t.ws, M);
    X = S;
  }
  template <int W>
  static __device__ __forceinline__ void gs_last(Res<W>& X, Res<W>& Y, const Tw<W>& ninv, const Tw<W>& ninv_w1,
                                                 const Modulus<W>& M) {
    const Res<4> S = A::add(X, Y);
    Res<4> D = A::add(X, M.q8);
    u32 b;
    D = A::sub(D, Y, b);
    Res<4> x = A::shoup_mul(S, ninv.w, ninv.ws, M);
    Res<4> y = A::shoup_mul(D, ninv_w1.w, ninv_w1.ws, M);
    x = A::csub(A::csub(A::csub(x, M.q4), M.q2), M.q);
    y = A::csub(A::csub(A::csub(y, M.q4), M.q2), M.q);
    X = x;
    Y = y;
  }
  template <int W>
  static __device__ __forceinline__ Res<W> canon(const Res<W>& x, const Modulus<W>& M) {
    return A::csub(A::csub(A::csub(A::csub(x, M.q8), M.q4), M.q2), M.q);
  }
};

}  // namespace mw
