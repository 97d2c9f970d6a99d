// NTT butterflies on multi-word residues (SIMD-vectorized kernels, from
// arithmetic to cryptographic kernels: one modular multiplication, one
// addition and one subtraction each), with the lazy value ranges the tile
// engines rely on.  Pure register arithmetic on top of mw_arith.h, so the CPU
// emulation test can compile it for the host.
#pragma once

#include "mw_arith.h"

namespace mw {

// A twiddle factor and its Shoup companion floor(w * 2^(32W) / q).
template <int W>
struct Tw {
  u32 w[W];
  u32 ws[W];
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

// Canonical x mod q for x in [0, 16q).
// When q's top word q_top has at least 17 bits (M.est_ok), the quotient
// k = floor(x / q) <= 15 is estimated from x's top word t:
// k' = trunc(float(t) * r), with r < 1 / (q_top + 1) (set_quotient_estimate).
// - k' <= t / (q_top + 1) <= x / q, so k' <= k.
// - x / q - t / (q_top + 1) < 17 / q_top <= 2^-11.9, and the float roundings
//   lose less than 2^-15, so k <= k' + 1.
// Then x - k'q is in [0, 2q), and one conditional subtraction of q ends it:
// 19 word instructions for two words instead of the 32 of four conditional
// subtractions (8q, 4q, 2q, q), which remain for smaller moduli.
template <int W>
__device__ __forceinline__ Res<W> canon16(const Res<W>& x, const Modulus<W>& M) {
  if (M.est_ok) {
    const u32 k = (u32)((float)x.v[W - 1] * __builtin_bit_cast(float, M.est_rcp));
    u32 kq[W];
    u64 c = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const u64 t = mad(k, M.q[i], c);   // k < 16: no overflow, and k q < 2^(32W)
      kq[i] = (u32)t;
      c = t >> 32;
    }
    u32 borrow;
    return csub(sub(x, kq, borrow), M.q);
  }
  return csub(csub(csub(csub(x, M.q8), M.q4), M.q2), M.q);
}

// The butterflies as a policy type for the tile engines (the arithmetic
// variants of mw_ablation.h provide the same four functions).
struct NativeBfly {
  template <int W>
  static __device__ __forceinline__ void ct(Res<W>& X, Res<W>& Y, const Tw<W>& t, const Modulus<W>& M) {
    ct_bfly(X, Y, t, M);
  }
  template <int W>
  static __device__ __forceinline__ void gs(Res<W>& X, Res<W>& Y, const Tw<W>& t, const Modulus<W>& M) {
    gs_bfly(X, Y, t, M);
  }
  template <int W>
  static __device__ __forceinline__ void gs_last(Res<W>& X, Res<W>& Y, const Tw<W>& ninv, const Tw<W>& ninv_w1,
                                                 const Modulus<W>& M) {
    gs_bfly_last(X, Y, ninv, ninv_w1, M);
  }
  template <int W>
  static __device__ __forceinline__ Res<W> canon(const Res<W>& x, const Modulus<W>& M) {
    return canon16(x, M);
  }
};

}  // namespace mw
