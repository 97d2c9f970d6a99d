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

template <int W>
__device__ __forceinline__ Res<W> canon16(const Res<W>& x, const Modulus<W>& M) {
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
