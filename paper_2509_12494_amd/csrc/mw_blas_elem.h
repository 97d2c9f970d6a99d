// Element-wise modular BLAS operations on one residue (Background,
// polynomial operations as BLAS), shared by the streaming BLAS kernels and
// the serving runtime's resident request loop.
#pragma once
#include "mw_arith.h"

namespace mw {

enum BlasOp { OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_AXPY = 3 };

template <int W>
struct Scalar {
  u32 w[W];
  u32 ws[W];
};

// NORM: products reduce on the scaled modulus (a modulus below the top of its
// width class; a kernel of its own, so the full-width one keeps its code).
// KARA: the full product by one level of Karatsuba (Eq. mulk).
template <int W, int OP, bool NORM, bool KARA = false>
__device__ __forceinline__ Res<W> blas_elem(const Res<W>& a, const Res<W>& b, const Modulus<W>& M,
                                           const Scalar<W>& s) {
  if constexpr (OP == OP_ADD) {
    return addmod(a, b, M);
  } else if constexpr (OP == OP_SUB) {
    return submod(a, b, M);
  } else if constexpr (OP == OP_MUL) {
    return barrett_mul_t<W, NORM, KARA>(a, b, M);
  } else {
    // a = x, b = y: alpha*x in [0, 6q), + y in [0, 7q) -> canonical
    Res<W> t = shoup_mul(a, s.w, s.ws, M);
    t = add(t, b);
    t = csub(t, M.q4);
    t = csub(t, M.q2);
    return csub(t, M.q);
  }
}

}  // namespace mw
