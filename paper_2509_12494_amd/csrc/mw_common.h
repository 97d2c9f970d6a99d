// Host-side helpers shared by the BLAS and NTT entry points: modulus checks and
// the per-modulus constants passed to the kernels.
#pragma once
#include <stdint.h>

#include "../../include/mwntt.h"
#include "mw_arith.h"
#include "mw_host_math.h"
#include "mw_host_wide.h"

namespace mw {

// Width rules (see mwntt.h): limbs == 1 -> odd 3 <= q < 2^60, limbs == 2 ->
// 2^60 <= q < 2^124, limbs == 4 -> 2^124 <= q < 2^252.  Every operation
// (Barrett multiplication included) takes any odd modulus of its class.
inline int check_modulus(const uint64_t* q, uint32_t limbs) {
  if (!q || (limbs != 1 && limbs != 2 && limbs != 4)) return MW_EINVAL;
  if (limbs == 4) {
    const mwhost::U256 Q = mwhost::u256_from_words(q, 4);
    const int b = mwhost::bitlen(Q);
    if (!(Q.w[0] & 1) || b > 252 || b < 125) return MW_EMODULUS;
    return MW_OK;
  }
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  int b = mwhost::bitlen(Q);
  if (!(Q & 1) || Q < 3) return MW_EMODULUS;
  if (limbs == 1) {
    if (b > 60) return MW_EMODULUS;
  } else {
    if (b > 124 || b < 61) return MW_EMODULUS;
  }
  return MW_OK;
}

template <int W>
inline void put_words(mwhost::u128 v, u32 (&out)[W]) {
  for (int i = 0; i < W; ++i) out[i] = (u32)(v >> (32 * i));
}

// The reciprocal canon16 estimates a quotient with: r = (1 - 2^-20) / (q_top + 1)
// in double, rounded to float (at most 2^-24 up), so r < 1 / (q_top + 1).
// Used when q's top word q_top has at least 17 bits.
template <int W>
inline void set_quotient_estimate(Modulus<W>& M) {
  const u32 top = M.q[W - 1];
  M.est_ok = top >= (1u << 16) ? 1u : 0u;
  const float r = (float)((1.0 - 1.0 / (1 << 20)) / ((double)top + 1.0));
  M.est_rcp = M.est_ok ? __builtin_bit_cast(u32, r) : 0u;
}

template <int W>
inline void make_modulus(const uint64_t* q, uint32_t limbs, Modulus<W>& M) {
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  int b = mwhost::bitlen(Q);
  put_words<W>(Q, M.q);
  put_words<W>(2 * Q, M.q2);
  put_words<W>(4 * Q, M.q4);
  put_words<W>(8 * Q, M.q8);
  put_words<W>((mwhost::u128)0 - Q, M.negq);  // 2^(32W) - q (W = 4: 2^128 - q)
  // Barrett on q' = q * 2^s with bitlen(q') = 32W - 4
  const int T = barrett_bits<W>();
  const mwhost::u128 Qn = Q << (T - b);
  put_words<W>(Qn, M.qn);
  put_words<W>(2 * Qn, M.qn2);
  put_words<W>(mwhost::pow2_div(2 * T, Qn), M.mu);
  M.bits = (u32)b;
  M.shift = (u32)(T - b);
  set_quotient_estimate(M);
}

template <int W>
inline void put_words(const mwhost::U256& v, u32 (&out)[W]) {
  for (int i = 0; i < W; ++i) out[i] = (u32)(v.w[i / 2] >> (32 * (i % 2)));
}

// Four-word moduli (W = 8 32-bit words).
inline void make_modulus(const uint64_t* q, Modulus<8>& M) {
  const mwhost::U256 Q = mwhost::u256_from_words(q, 4);
  const int b = mwhost::bitlen(Q);
  put_words<8>(Q, M.q);
  put_words<8>(mwhost::shl(Q, 1), M.q2);
  put_words<8>(mwhost::shl(Q, 2), M.q4);
  put_words<8>(mwhost::shl(Q, 3), M.q8);            // 8q < 2^255
  put_words<8>(mwhost::sub(mwhost::u256(0), Q), M.negq);  // 2^256 - q
  const int T = barrett_bits<8>();
  const mwhost::U256 Qn = mwhost::shl_any(Q, T - b);
  put_words<8>(Qn, M.qn);
  put_words<8>(mwhost::shl(Qn, 1), M.qn2);                 // 2q' < 2^253
  put_words<8>(mwhost::pow2_div(2 * T, Qn), M.mu);
  M.bits = (u32)b;
  M.shift = (u32)(T - b);
  set_quotient_estimate(M);
}

inline int make_scalar(const uint64_t* w, const uint64_t* q, u32 (&wv)[8], u32 (&ws)[8]) {
  const mwhost::U256 Q = mwhost::u256_from_words(q, 4), Wv = mwhost::u256_from_words(w, 4);
  if (!(Wv < Q)) return MW_EINVAL;
  put_words<8>(Wv, wv);
  put_words<8>(mwhost::shoup(Wv, Q, 256), ws);
  return MW_OK;
}

// Constant multiplier and its Shoup companion floor(w * 2^(32W) / q).
template <int W>
inline int make_scalar(const uint64_t* w, const uint64_t* q, uint32_t limbs, u32 (&wv)[W], u32 (&ws)[W]) {
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  mwhost::u128 Wv = mwhost::from_words(w, limbs);
  if (Wv >= Q) return MW_EINVAL;
  put_words<W>(Wv, wv);
  put_words<W>(mwhost::shoup(Wv, Q, 32 * W), ws);
  return MW_OK;
}

}  // namespace mw
