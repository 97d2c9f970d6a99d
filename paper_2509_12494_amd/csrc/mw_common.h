// Host-side helpers shared by the BLAS and NTT entry points: modulus checks and
// the per-modulus constants passed to the kernels.
#pragma once
#include <stdint.h>

#include "../../include/mwntt.h"
#include "mw_arith.h"
#include "mw_host_math.h"

namespace mw {

// Width rules (see mwntt.h): limbs == 1 -> q < 2^60, limbs == 2 -> 2^60 <= q < 2^124.
// Barrett multiplication additionally needs bitlen(q) >= 33 (limbs 1) or
// >= 97 (limbs 2).
inline int check_modulus(const uint64_t* q, uint32_t limbs, bool barrett) {
  if (!q || (limbs != 1 && limbs != 2)) return MW_EINVAL;
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  int b = mwhost::bitlen(Q);
  if (!(Q & 1) || Q < 3) return MW_EMODULUS;
  if (limbs == 1) {
    if (b > 60) return MW_EMODULUS;
    if (barrett && b < 33) return MW_EMODULUS;
  } else {
    if (b > 124 || b < 61) return MW_EMODULUS;
    if (barrett && b < 97) return MW_EMODULUS;
  }
  return MW_OK;
}

template <int W>
inline void put_words(mwhost::u128 v, u32 (&out)[W]) {
  for (int i = 0; i < W; ++i) out[i] = (u32)(v >> (32 * i));
}

template <int W>
inline void make_modulus(const uint64_t* q, uint32_t limbs, Modulus<W>& M) {
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  int b = mwhost::bitlen(Q);
  put_words<W>(Q, M.q);
  put_words<W>(2 * Q, M.q2);
  put_words<W>(4 * Q, M.q4);
  put_words<W>(8 * Q, M.q8);
  put_words<W>(mwhost::pow2_div(2 * b, Q), M.mu);
  put_words<W>((mwhost::u128)0 - Q, M.negq);  // 2^(32W) - q (W = 4: 2^128 - q)
  M.bits = (u32)b;
  M.pad_[0] = M.pad_[1] = M.pad_[2] = 0;
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
