// Element-wise modular BLAS over Z_q (Background, polynomial operations as
// BLAS): c = a + b, c = a - b, c = a * b (Barrett, Eq. barrett) and
// y = alpha*x + y (Shoup multiplication by the constant alpha).
//
// These are streaming kernels bound by HBM bandwidth (124-bit add/sub/axpy) or
// close to the VALU ridge (124- and 252-bit mulmod).  A block of 256 lanes
// handles VEC residues per lane per chunk with 16-byte vector accesses; the
// grid covers every chunk (a grid-stride loop only past 2^30 blocks), and a
// guarded path handles the ragged tail.
//
// Access form per width, from a triad probe (two streams read, one written,
// the 2^24-residue workload) on MI355X:
//   one word   8-byte residues, non-temporal stores             7.27 TB/s
//   two words  16-byte residues, non-temporal loads, 2 per lane 7.03 TB/s
//              (non-temporal loads and stores: 6.52; a 2048-block grid with
//              a stride loop: 6.22)
//   four words 32-byte residues read as two 16-byte halves by one lane touch
//              twice the cache lines per instruction (5.5-5.8 TB/s); the
//              block instead moves its residues as coalesced 16-byte units
//              through LDS and each lane takes its residue from there:
//              6.97 TB/s with non-temporal loads.
#include <hip/hip_runtime.h>

#include "mw_arith.h"
#include "mw_blas_elem.h"
#include "mw_common.h"
#include "mw_tuned.h"
#include "mw_validate.h"

#include <atomic>

namespace mw {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Loads and stores of the main streaming loop, per width (see the access
// forms above; four-word residues go through LDS instead).
template <int W>
struct Stream;
template <>
struct Stream<2> {
  static constexpr int VEC = 4;
  __device__ static __forceinline__ Res<2> load(const Res<2>* p) { return ResIO<2>::load(p); }
  __device__ static __forceinline__ void store(Res<2>* p, const Res<2>& r) {
    const u32x2 v = {r.v[0], r.v[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x2*>(p));
  }
};
template <>
struct Stream<4> {
  static constexpr int VEC = 2;
  __device__ static __forceinline__ Res<4> load(const Res<4>* p) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    Res<4> r;
    r.v[0] = v.x; r.v[1] = v.y; r.v[2] = v.z; r.v[3] = v.w;
    return r;
  }
  __device__ static __forceinline__ void store(Res<4>* p, const Res<4>& r) { ResIO<4>::store(p, r); }
};
template <>
struct Stream<8> {
  static constexpr int VEC = 1;
};

constexpr int kBlasThreads = 256;

// One chunk of four-word residues through LDS: the block's 2*VEC*256 16-byte
// units of a and of b are loaded coalesced (non-temporal) into LDS, each lane
// takes its residue(s) from there, writes the result over a's slots, and the
// block stores the units coalesced.
template <int OP, int VEC, bool NORM, bool KARA>
__device__ __forceinline__ void blas_chunk8(Res<8>* c, const Res<8>* a, const Res<8>* b, u64 base_res,
                                            const Modulus<8>& M, const Scalar<8>& s, u32x4* la, u32x4* lb) {
  const u32 t = threadIdx.x;
  const u32x4* ga = reinterpret_cast<const u32x4*>(a + base_res);
  const u32x4* gb = reinterpret_cast<const u32x4*>(b + base_res);
  u32x4 va[2 * VEC], vb[2 * VEC];
#pragma unroll
  for (int k = 0; k < 2 * VEC; ++k) {
    va[k] = __builtin_nontemporal_load(ga + t + k * kBlasThreads);
    vb[k] = __builtin_nontemporal_load(gb + t + k * kBlasThreads);
  }
#pragma unroll
  for (int k = 0; k < 2 * VEC; ++k) {
    la[t + k * kBlasThreads] = va[k];
    lb[t + k * kBlasThreads] = vb[k];
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const u32 e = t + v * kBlasThreads;
    const Res<8> x = ResIO<8>::load(la + 2 * e), y = ResIO<8>::load(lb + 2 * e);
    ResIO<8>::store(la + 2 * e, blas_elem<8, OP, NORM, KARA>(x, y, M, s));
  }
  __syncthreads();
  u32x4* gc = reinterpret_cast<u32x4*>(c + base_res);
#pragma unroll
  for (int k = 0; k < 2 * VEC; ++k) gc[t + k * kBlasThreads] = la[t + k * kBlasThreads];
  __syncthreads();                                 // the next chunk reuses the slots
}

template <int W, int OP, int VEC, bool NORM, bool KARA>
__global__ __launch_bounds__(kBlasThreads) void blas_kernel(Res<W>* c, const Res<W>* a, const Res<W>* b, u64 n,
                                                           Modulus<W> M, Scalar<W> s) {
  const u64 chunk = (u64)VEC * kBlasThreads;
  const u64 nfull = n / chunk;
  if constexpr (W == 8) {
    __shared__ u32x4 la[2 * VEC * kBlasThreads];
    __shared__ u32x4 lb[2 * VEC * kBlasThreads];
    for (u64 blk = blockIdx.x; blk < nfull; blk += gridDim.x)
      blas_chunk8<OP, VEC, NORM, KARA>(c, a, b, blk * chunk, M, s, la, lb);
  } else {
    for (u64 blk = blockIdx.x; blk < nfull; blk += gridDim.x) {
      const u64 base = blk * chunk + threadIdx.x;
      Res<W> x[VEC], y[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        x[v] = Stream<W>::load(a + base + (u64)v * kBlasThreads);
        y[v] = Stream<W>::load(b + base + (u64)v * kBlasThreads);
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v)
        Stream<W>::store(c + base + (u64)v * kBlasThreads, blas_elem<W, OP, NORM, KARA>(x[v], y[v], M, s));
    }
  }
  // ragged tail: residues [nfull*chunk, n), handled by the one block whose
  // turn comes next in the grid-stride order
  if (blockIdx.x == (unsigned)(nfull % gridDim.x)) {
    for (u64 i = nfull * chunk + threadIdx.x; i < n; i += blockDim.x) {
      Res<W> x = ResIO<W>::load(a + i), y = ResIO<W>::load(b + i);
      ResIO<W>::store(c + i, blas_elem<W, OP, NORM, KARA>(x, y, M, s));
    }
  }
}

// Product kernel of vec_mulmod per width (index: limbs 1, 2, 4 -> 0, 1, 2):
// 0 schoolbook, 1 Karatsuba.  Starts from the measured choice (mw_tuned.h);
// vec_mulmod_set_product changes it for later calls.
std::atomic<uint32_t> g_kara[3] = {{tuned_karatsuba(1)}, {tuned_karatsuba(2)}, {tuned_karatsuba(4)}};

inline int width_slot(uint32_t limbs) { return limbs == 1 ? 0 : (limbs == 2 ? 1 : (limbs == 4 ? 2 : -1)); }

template <int W, int OP, bool NORM, bool KARA>
static void launch_blas_kernel(unsigned grid, hipStream_t stream, void* d_c, const void* d_a, const void* d_b,
                               size_t n, const Modulus<W>& M, const Scalar<W>& s) {
  hipLaunchKernelGGL((blas_kernel<W, OP, Stream<W>::VEC, NORM, KARA>), dim3(grid), dim3(kBlasThreads), 0, stream,
                     reinterpret_cast<Res<W>*>(d_c), reinterpret_cast<const Res<W>*>(d_a),
                     reinterpret_cast<const Res<W>*>(d_b), (u64)n, M, s);
}

template <int W, int OP>
static int launch_blas(void* d_c, const void* d_a, const void* d_b, size_t n, const Modulus<W>& M,
                       const Scalar<W>& s, hipStream_t stream) {
  const u64 chunk = (u64)Stream<W>::VEC * kBlasThreads;
  const u64 chunks = (n + chunk - 1) / chunk;
  // one block per chunk; past 2^30 blocks the grid-stride loop iterates
  u64 grid = chunks < (u64(1) << 30) ? chunks : (u64(1) << 30);
  if (grid == 0) grid = 1;
  const unsigned g = (unsigned)grid;
  if constexpr (OP == OP_MUL) {
    const bool kara = g_kara[width_slot(W / 2)].load(std::memory_order_relaxed) != 0;
    if (M.shift != 0) {
      if (kara) launch_blas_kernel<W, OP, true, true>(g, stream, d_c, d_a, d_b, n, M, s);
      else launch_blas_kernel<W, OP, true, false>(g, stream, d_c, d_a, d_b, n, M, s);
    } else {
      if (kara) launch_blas_kernel<W, OP, false, true>(g, stream, d_c, d_a, d_b, n, M, s);
      else launch_blas_kernel<W, OP, false, false>(g, stream, d_c, d_a, d_b, n, M, s);
    }
  } else {
    launch_blas_kernel<W, OP, false, false>(g, stream, d_c, d_a, d_b, n, M, s);
  }
  return hipGetLastError() == hipSuccess ? MW_OK : MW_EDEVICE;
}

// Per-thread memo of the last modulus (and axpy scalar) of each width: the
// constants (Barrett mu and the Shoup companion come from bitwise long
// division) are the same on every call of a loop over one modulus.
template <int W>
struct ModMemo {
  uint64_t q[4] = {0, 0, 0, 0};
  Modulus<W> M{};
  bool valid = false;
  uint64_t alpha[4] = {0, 0, 0, 0};
  Scalar<W> sc{};
  bool sc_valid = false;
};

static bool same_words(const uint64_t* a, const uint64_t* b, uint32_t limbs) {
  for (uint32_t i = 0; i < limbs; ++i)
    if (a[i] != b[i]) return false;
  return true;
}

template <int W>
static const Modulus<W>& memo_modulus(const uint64_t* q, uint32_t limbs) {
  thread_local ModMemo<W> m;
  if (!m.valid || !same_words(m.q, q, limbs)) {
    if constexpr (W == 8) make_modulus(q, m.M);
    else make_modulus<W>(q, limbs, m.M);
    for (uint32_t i = 0; i < 4; ++i) m.q[i] = i < limbs ? q[i] : 0;
    m.valid = true;
    m.sc_valid = false;
  }
  return m.M;
}

// alpha and its Shoup companion, memoized per thread by (q, alpha)
template <int W>
static int memo_scalar(const uint64_t* alpha, const uint64_t* q, uint32_t limbs, Scalar<W>& out) {
  thread_local ModMemo<W> m;   // separate memo: keyed by (q, alpha)
  if (!m.sc_valid || !same_words(m.q, q, limbs) || !same_words(m.alpha, alpha, limbs)) {
    Scalar<W> sc = {};
    int st;
    if constexpr (W == 8) st = make_scalar(alpha, q, sc.w, sc.ws);
    else st = make_scalar(alpha, q, limbs, sc.w, sc.ws);
    if (st != MW_OK) return st;
    for (uint32_t i = 0; i < 4; ++i) {
      m.q[i] = i < limbs ? q[i] : 0;
      m.alpha[i] = i < limbs ? alpha[i] : 0;
    }
    m.sc = sc;
    m.sc_valid = true;
  }
  out = m.sc;
  return MW_OK;
}

// report: a pending validate-mode violation is returned by this call (the
// public entry points); the serving runtime leaves it for mw_check.
template <int OP>
static int blas_dispatch(void* d_c, const void* d_a, const void* d_b, size_t n, const uint64_t* q,
                         uint32_t limbs, const uint64_t* alpha, void* stream, bool report = true) {
  if (!q || (limbs != 1 && limbs != 2 && limbs != 4)) return MW_EINVAL;
  if (n == 0) return MW_OK;
  if (!d_c || !d_a || !d_b) return MW_EINVAL;
  if (n > ((size_t)1 << 40)) return MW_EINVAL;
  int st = check_modulus(q, limbs);
  if (st != MW_OK) return st;
  if (OP == OP_AXPY && !alpha) return MW_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (validate_on()) {
    if (report && (st = validate_take()) != MW_OK) return st;
    if ((st = validate_input(d_a, n, q, limbs, s)) != MW_OK) return st;
    if ((st = validate_input(d_b, n, q, limbs, s)) != MW_OK) return st;
  }
  if (limbs == 4) {
    Scalar<8> sc = {};
    if (OP == OP_AXPY && memo_scalar<8>(alpha, q, limbs, sc) != MW_OK) return MW_EINVAL;
    return launch_blas<8, OP>(d_c, d_a, d_b, n, memo_modulus<8>(q, limbs), sc, s);
  } else if (limbs == 2) {
    Scalar<4> sc = {};
    if (OP == OP_AXPY && memo_scalar<4>(alpha, q, limbs, sc) != MW_OK) return MW_EINVAL;
    return launch_blas<4, OP>(d_c, d_a, d_b, n, memo_modulus<4>(q, limbs), sc, s);
  } else {
    Scalar<2> sc = {};
    if (OP == OP_AXPY && memo_scalar<2>(alpha, q, limbs, sc) != MW_OK) return MW_EINVAL;
    return launch_blas<2, OP>(d_c, d_a, d_b, n, memo_modulus<2>(q, limbs), sc, s);
  }
}

// Internal entry for the serving runtime: op 0..3 = add, sub, mul, axpy
// (axpy: c = alpha*a + b, c may differ from b).
int blas_launch(int op, void* d_c, const void* d_a, const void* d_b, size_t n, const uint64_t* q, uint32_t limbs,
                const uint64_t* alpha, void* stream) {
  switch (op) {
    case OP_ADD: return blas_dispatch<OP_ADD>(d_c, d_a, d_b, n, q, limbs, nullptr, stream, false);
    case OP_SUB: return blas_dispatch<OP_SUB>(d_c, d_a, d_b, n, q, limbs, nullptr, stream, false);
    case OP_MUL: return blas_dispatch<OP_MUL>(d_c, d_a, d_b, n, q, limbs, nullptr, stream, false);
    case OP_AXPY: return blas_dispatch<OP_AXPY>(d_c, d_a, d_b, n, q, limbs, alpha, stream, false);
    default: return MW_EINVAL;
  }
}

}  // namespace mw

using namespace mw;

extern "C" int vec_addmod(void* d_c, const void* d_a, const void* d_b, size_t n, const uint64_t* q,
                          uint32_t limbs, void* stream) {
  return blas_dispatch<OP_ADD>(d_c, d_a, d_b, n, q, limbs, nullptr, stream);
}

extern "C" int vec_submod(void* d_c, const void* d_a, const void* d_b, size_t n, const uint64_t* q,
                          uint32_t limbs, void* stream) {
  return blas_dispatch<OP_SUB>(d_c, d_a, d_b, n, q, limbs, nullptr, stream);
}

extern "C" int vec_mulmod(void* d_c, const void* d_a, const void* d_b, size_t n, const uint64_t* q,
                          uint32_t limbs, void* stream) {
  return blas_dispatch<OP_MUL>(d_c, d_a, d_b, n, q, limbs, nullptr, stream);
}

extern "C" int vec_axpymod(void* d_y, const uint64_t* alpha, const void* d_x, size_t n, const uint64_t* q,
                           uint32_t limbs, void* stream) {
  // y <- alpha*x + y: the kernel reads (a = x, b = y) and writes c = y
  return blas_dispatch<OP_AXPY>(d_y, d_x, d_y, n, q, limbs, alpha, stream);
}

extern "C" int vec_mulmod_set_product(uint32_t limbs, uint32_t karatsuba) {
  const int k = width_slot(limbs);
  if (k < 0 || karatsuba > 1) return MW_EINVAL;
  g_kara[k].store(karatsuba, std::memory_order_relaxed);
  return MW_OK;
}

extern "C" int vec_mulmod_get_product(uint32_t limbs, uint32_t* karatsuba) {
  const int k = width_slot(limbs);
  if (k < 0 || !karatsuba) return MW_EINVAL;
  *karatsuba = g_kara[k].load(std::memory_order_relaxed);
  return MW_OK;
}

extern "C" int mw_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return MW_OK;
  if (!dst || !src) return MW_EINVAL;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? MW_OK
             : MW_EDEVICE;
}
