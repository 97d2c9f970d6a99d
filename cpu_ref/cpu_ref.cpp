// Plain scalar CPU baseline of the hot path, for measurement beside the GPU:
// negacyclic NTT (forward and inverse) and the modular BLAS operations over
// moduli of one, two or four 64-bit words, in the paper's scalar double-word
// style (Background, double-word arithmetic: 64-bit words with the compiler's
// unsigned __int128 holding the results of 64-bit adds and multiplies, so it
// can use add-with-carry), with
//   * addition and subtraction by one conditional correction (Eq. saddmod,
//     ssubmod),
//   * multiplication as the schoolbook product of the words (Eq. muls) and
//     Barrett reduction with mu = floor(2^k / q), k = 2 bitlen(q) (Eq.
//     barrett; 2^(k/2) > q as the paper requires), one final correction,
//   * iterative radix-2 transforms: Cooley-Tukey forward with the powers of
//     psi in bit-reversed order (the negacyclic twist merged into the
//     butterflies), Gentleman-Sande inverse, every value canonical after
//     every butterfly.
// No SIMD intrinsics and no lazy reduction: it is the plain baseline, not a
// tuned CPU kernel.  Nothing in the GPU library calls it.
//
// Threads: a transform call splits its batch over threads, a BLAS call its
// vector in contiguous chunks; threads = 0 means every hardware thread.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <thread>
#include <vector>

typedef unsigned __int128 u128;

namespace {

enum { CR_OK = 0, CR_EINVAL = -1, CR_EMODULUS = -2, CR_ENOMEM = -3, CR_EROOT = -4 };
enum { OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_AXPY = 3 };

// A residue: L 64-bit words, least significant first.
template <int L>
struct Num {
  uint64_t w[L];
};

template <int L>
inline bool geq(const uint64_t* a, const uint64_t* b) {
  for (int i = L - 1; i >= 0; --i)
    if (a[i] != b[i]) return a[i] > b[i];
  return true;
}

// r = a + b over n words, returns the carry out
inline uint64_t add_n(uint64_t* r, const uint64_t* a, const uint64_t* b, int n) {
  u128 c = 0;
  for (int i = 0; i < n; ++i) {
    c += (u128)a[i] + b[i];
    r[i] = (uint64_t)c;
    c >>= 64;
  }
  return (uint64_t)c;
}

// r = a - b over n words, returns the borrow out
inline uint64_t sub_n(uint64_t* r, const uint64_t* a, const uint64_t* b, int n) {
  uint64_t borrow = 0;
  for (int i = 0; i < n; ++i) {
    const u128 d = (u128)a[i] - b[i] - borrow;
    r[i] = (uint64_t)d;
    borrow = (uint64_t)(d >> 64) & 1;
  }
  return borrow;
}

// r[0 .. na+nb) = a * b, schoolbook: one 64 x 64 -> 128-bit product per
// pair of words, rows accumulated with their carries
inline void mul_n(uint64_t* r, const uint64_t* a, int na, const uint64_t* b, int nb) {
  for (int i = 0; i < na + nb; ++i) r[i] = 0;
  for (int i = 0; i < na; ++i) {
    u128 carry = 0;
    for (int j = 0; j < nb; ++j) {
      const u128 t = (u128)a[i] * b[j] + r[i + j] + carry;
      r[i + j] = (uint64_t)t;
      carry = t >> 64;
    }
    r[i + nb] = (uint64_t)carry;
  }
}

// r[0 .. rn) = the low rn words of a >> s (a has n words)
inline void shr_n(uint64_t* r, int rn, const uint64_t* a, int n, int s) {
  const int ws = s / 64, bs = s % 64;
  for (int i = 0; i < rn; ++i) {
    const uint64_t lo = i + ws < n ? a[i + ws] >> bs : 0;
    const uint64_t hi = (bs && i + ws + 1 < n) ? a[i + ws + 1] << (64 - bs) : 0;
    r[i] = lo | hi;
  }
}

inline int bitlen_n(const uint64_t* a, int n) {
  for (int i = n - 1; i >= 0; --i)
    if (a[i]) return 64 * i + 64 - __builtin_clzll(a[i]);
  return 0;
}

// The modulus and its Barrett constant mu = floor(2^k / q), k = 2 bitlen(q).
template <int L>
struct Mod {
  uint64_t q[L];
  uint64_t mu[L + 1];   // bitlen(mu) = bitlen(q) + 1 at most
  int k;
};

// floor(2^k / q) by binary long division (setup only)
template <int L>
void barrett_mu(Mod<L>& M) {
  const int b = bitlen_n(M.q, L);
  M.k = 2 * b;
  uint64_t rem[L + 1] = {0};
  uint64_t quo[L + 1] = {0};
  uint64_t qq[L + 1] = {0};
  for (int i = 0; i < L; ++i) qq[i] = M.q[i];
  for (int bit = M.k; bit >= 0; --bit) {
    // rem = 2 rem + (bit == k)
    uint64_t carry = bit == M.k ? 1 : 0;
    for (int i = 0; i <= L; ++i) {
      const uint64_t nc = rem[i] >> 63;
      rem[i] = (rem[i] << 1) | carry;
      carry = nc;
    }
    if (geq<L + 1>(rem, qq)) {
      sub_n(rem, rem, qq, L + 1);
      if (bit < 64 * (L + 1)) quo[bit / 64] |= uint64_t(1) << (bit % 64);
    }
  }
  for (int i = 0; i <= L; ++i) M.mu[i] = quo[i];
}

template <int L>
inline void addmod(uint64_t* c, const uint64_t* a, const uint64_t* b, const Mod<L>& M) {
  uint64_t s[L];
  const uint64_t carry = add_n(s, a, b, L);
  if (carry || geq<L>(s, M.q)) sub_n(s, s, M.q, L);
  memcpy(c, s, sizeof(s));
}

template <int L>
inline void submod(uint64_t* c, const uint64_t* a, const uint64_t* b, const Mod<L>& M) {
  uint64_t d[L];
  if (sub_n(d, a, b, L)) add_n(d, d, M.q, L);
  memcpy(c, d, sizeof(d));
}

// c = a b - floor(a b mu / 2^k) q, then one conditional subtraction
template <int L>
inline void mulmod(uint64_t* c, const uint64_t* a, const uint64_t* b, const Mod<L>& M) {
  uint64_t x[2 * L];
  mul_n(x, a, L, b, L);
  uint64_t t[3 * L + 1];
  mul_n(t, x, 2 * L, M.mu, L + 1);
  uint64_t qh[L + 1];
  shr_n(qh, L + 1, t, 3 * L + 1, M.k);      // < 2^(bitlen(q) + 1): L + 1 words hold it
  uint64_t p[2 * L + 1];
  mul_n(p, qh, L + 1, M.q, L);
  uint64_t r[L + 1];
  sub_n(r, x, p, L + 1);                    // exact: 0 <= x - qh q < 2q
  if (r[L] || geq<L>(r, M.q)) sub_n(r, r, M.q, L);
  memcpy(c, r, sizeof(uint64_t) * L);
}

template <int L>
void powmod(uint64_t* r, const uint64_t* base, const uint64_t* e, int ebits, const Mod<L>& M) {
  uint64_t acc[L] = {0};
  acc[0] = 1;
  for (int i = ebits - 1; i >= 0; --i) {
    mulmod<L>(acc, acc, acc, M);
    if ((e[i / 64] >> (i % 64)) & 1) mulmod<L>(acc, acc, base, M);
  }
  memcpy(r, acc, sizeof(acc));
}

inline uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

// Precomputed tables of a transform size: psi^bitrev(i) and psi^-bitrev(i)
// for i < N, N^-1.
template <int L>
struct Plan {
  Mod<L> M;
  uint32_t log2n;
  std::vector<Num<L>> fwd, inv;
  Num<L> ninv;
};

template <int L>
bool is_minus_one(const uint64_t* a, const Mod<L>& M) {
  uint64_t t[L];
  memcpy(t, a, sizeof(t));
  uint64_t one[L] = {0};
  one[0] = 1;
  add_n(t, t, one, L);
  return !memcmp(t, M.q, sizeof(t));
}

// The smallest primitive 2N-th root of unity mod the prime q: a quadratic
// non-residue g (Euler's criterion) gives psi0 = g^((q-1)/2N), whose odd
// powers are all the primitive 2N-th roots.
template <int L>
int canonical_root(const Mod<L>& M, uint32_t log2n, uint64_t* out) {
  uint64_t qm1[L];
  memcpy(qm1, M.q, sizeof(qm1));
  qm1[0] -= 1;   // q odd
  const int qb = bitlen_n(M.q, L);
  uint64_t e_half[L], e_root[L];
  shr_n(e_half, L, qm1, L, 1);
  shr_n(e_root, L, qm1, L, (int)log2n + 1);
  uint64_t g[L] = {0};
  uint64_t t[L];
  for (g[0] = 2;; ++g[0]) {
    powmod<L>(t, g, e_half, qb, M);
    if (is_minus_one<L>(t, M)) break;
    if (g[0] > 100000) return CR_EROOT;
  }
  uint64_t psi0[L];
  powmod<L>(psi0, g, e_root, qb, M);
  uint64_t n_e[L] = {0};
  n_e[0] = uint64_t(1) << log2n;
  powmod<L>(t, psi0, n_e, 64, M);
  if (!is_minus_one<L>(t, M)) return CR_EROOT;
  uint64_t best[L], cur[L], sq[L];
  memcpy(best, psi0, sizeof(best));
  memcpy(cur, psi0, sizeof(cur));
  mulmod<L>(sq, psi0, psi0, M);
  for (uint64_t i = 1; i < (uint64_t(1) << log2n); ++i) {
    mulmod<L>(cur, cur, sq, M);
    if (!geq<L>(cur, best)) memcpy(best, cur, sizeof(best));
  }
  memcpy(out, best, sizeof(best));
  return CR_OK;
}

template <int L>
int make_plan(Plan<L>& P, const uint64_t* psi) {
  const uint32_t n = 1u << P.log2n;
  uint64_t p[L];
  memcpy(p, psi, sizeof(p));
  uint64_t t[L];
  uint64_t n_e[L] = {0};
  n_e[0] = n;
  powmod<L>(t, p, n_e, 64, P.M);
  if (!is_minus_one<L>(t, P.M)) return CR_EROOT;
  // psi^-1 = psi^(2N - 1)
  uint64_t pinv[L], e[L] = {0};
  e[0] = 2 * (uint64_t)n - 1;
  powmod<L>(pinv, p, e, 64, P.M);
  std::vector<Num<L>> pw(n), pwi(n);
  uint64_t cur[L] = {0}, curi[L] = {0};
  cur[0] = curi[0] = 1;
  for (uint32_t i = 0; i < n; ++i) {
    memcpy(pw[i].w, cur, sizeof(cur));
    memcpy(pwi[i].w, curi, sizeof(curi));
    mulmod<L>(cur, cur, p, P.M);
    mulmod<L>(curi, curi, pinv, P.M);
  }
  P.fwd.resize(n);
  P.inv.resize(n);
  for (uint32_t i = 0; i < n; ++i) {
    P.fwd[i] = pw[bitrev(i, P.log2n)];
    P.inv[i] = pwi[bitrev(i, P.log2n)];
  }
  // N^-1 = (q - (q - 1) / N) since N divides q - 1
  uint64_t qm1[L], k[L];
  memcpy(qm1, P.M.q, sizeof(qm1));
  qm1[0] -= 1;
  shr_n(k, L, qm1, L, (int)P.log2n);
  sub_n(P.ninv.w, P.M.q, k, L);
  return CR_OK;
}

// Forward: natural order in, natural order out.  Cooley-Tukey stages with
// twiddle psi^bitrev(m + i) leave A[bitrev(i)] at i; one permutation pass
// restores natural order.
template <int L>
void forward(const Plan<L>& P, Num<L>* a, Num<L>* tmp) {
  const uint32_t n = 1u << P.log2n;
  for (uint32_t m = 1, t = n >> 1; m < n; m <<= 1, t >>= 1) {
    for (uint32_t i = 0; i < m; ++i) {
      const uint64_t* w = P.fwd[m + i].w;
      const uint32_t j1 = 2 * i * t;
      for (uint32_t j = j1; j < j1 + t; ++j) {
        uint64_t v[L];
        mulmod<L>(v, a[j + t].w, w, P.M);
        uint64_t u[L];
        memcpy(u, a[j].w, sizeof(u));
        addmod<L>(a[j].w, u, v, P.M);
        submod<L>(a[j + t].w, u, v, P.M);
      }
    }
  }
  for (uint32_t i = 0; i < n; ++i) tmp[bitrev(i, P.log2n)] = a[i];
  memcpy(a, tmp, sizeof(Num<L>) * n);
}

// Inverse: natural order in and out; Gentleman-Sande stages on the
// bit-reversed input, then the N^-1 scaling.
template <int L>
void inverse(const Plan<L>& P, Num<L>* a, Num<L>* tmp) {
  const uint32_t n = 1u << P.log2n;
  for (uint32_t i = 0; i < n; ++i) tmp[i] = a[bitrev(i, P.log2n)];
  memcpy(a, tmp, sizeof(Num<L>) * n);
  for (uint32_t m = n >> 1, t = 1; m >= 1; m >>= 1, t <<= 1) {   // m = N/2 .. 1
    for (uint32_t i = 0; i < m; ++i) {
      const uint64_t* w = P.inv[m + i].w;
      const uint32_t j1 = 2 * i * t;
      for (uint32_t j = j1; j < j1 + t; ++j) {
        uint64_t u[L], v[L];
        memcpy(u, a[j].w, sizeof(u));
        memcpy(v, a[j + t].w, sizeof(v));
        addmod<L>(a[j].w, u, v, P.M);
        uint64_t d[L];
        submod<L>(d, u, v, P.M);
        mulmod<L>(a[j + t].w, d, w, P.M);
      }
    }
  }
  for (uint32_t i = 0; i < n; ++i) mulmod<L>(a[i].w, a[i].w, P.ninv.w, P.M);
}

template <int L>
void blas(int op, Num<L>* c, const Num<L>* a, const Num<L>* b, uint64_t lo, uint64_t hi, const Mod<L>& M,
          const uint64_t* alpha) {
  for (uint64_t i = lo; i < hi; ++i) {
    switch (op) {
      case OP_ADD: addmod<L>(c[i].w, a[i].w, b[i].w, M); break;
      case OP_SUB: submod<L>(c[i].w, a[i].w, b[i].w, M); break;
      case OP_MUL: mulmod<L>(c[i].w, a[i].w, b[i].w, M); break;
      default: {
        uint64_t t[L];
        mulmod<L>(t, alpha, a[i].w, M);
        addmod<L>(c[i].w, t, b[i].w, M);
      }
    }
  }
}

uint32_t thread_count(uint32_t threads, uint64_t work) {
  uint32_t t = threads ? threads : std::max(1u, std::thread::hardware_concurrency());
  return (uint32_t)std::min<uint64_t>(t, std::max<uint64_t>(work, 1));
}

template <typename F>
void parallel(uint32_t nthreads, uint64_t work, F f) {
  if (nthreads <= 1) {
    f(0, work);
    return;
  }
  std::vector<std::thread> pool;
  pool.reserve(nthreads);
  for (uint32_t t = 0; t < nthreads; ++t) {
    const uint64_t lo = work * t / nthreads, hi = work * (t + 1) / nthreads;
    pool.emplace_back([=] { f(lo, hi); });
  }
  for (auto& th : pool) th.join();
}

template <int L>
int check_mod(const uint64_t* q, Mod<L>& M) {
  memcpy(M.q, q, sizeof(uint64_t) * L);
  const int b = bitlen_n(M.q, L);
  // classes as the GPU library's: 2..60, 61..124, 125..252 bits, odd
  const int lo = L == 1 ? 2 : (L == 2 ? 61 : 125), hi = L == 1 ? 60 : (L == 2 ? 124 : 252);
  if (!(M.q[0] & 1) || b < lo || b > hi || (L == 1 && M.q[0] < 3)) return CR_EMODULUS;
  barrett_mu<L>(M);
  return CR_OK;
}

struct PlanAny {
  uint32_t limbs;
  void* p;
};

template <int L>
int plan_create_t(PlanAny** out, uint32_t log2n, const uint64_t* q, const uint64_t* psi) {
  Plan<L>* P = new (std::nothrow) Plan<L>();
  if (!P) return CR_ENOMEM;
  P->log2n = log2n;
  int st = check_mod<L>(q, P->M);
  if (st == CR_OK) {
    if ((q[0] - 1) & ((uint64_t(2) << log2n) - 1)) st = CR_EMODULUS;   // q = 1 mod 2N
  }
  uint64_t root[L];
  if (st == CR_OK) {
    if (psi) memcpy(root, psi, sizeof(root));
    else st = canonical_root<L>(P->M, log2n, root);
  }
  if (st == CR_OK) st = make_plan<L>(*P, root);
  if (st != CR_OK) {
    delete P;
    return st;
  }
  PlanAny* A = new (std::nothrow) PlanAny{(uint32_t)L, P};
  if (!A) {
    delete P;
    return CR_ENOMEM;
  }
  *out = A;
  return CR_OK;
}

template <int L>
int ntt_t(PlanAny* A, uint64_t* out, const uint64_t* in, uint32_t batch, int inv, uint32_t threads) {
  const Plan<L>& P = *static_cast<Plan<L>*>(A->p);
  const uint64_t n = uint64_t(1) << P.log2n;
  if (out != in) memmove(out, in, sizeof(uint64_t) * L * n * batch);
  Num<L>* data = reinterpret_cast<Num<L>*>(out);
  parallel(thread_count(threads, batch), batch, [&](uint64_t lo, uint64_t hi) {
    std::vector<Num<L>> tmp(n);
    for (uint64_t b = lo; b < hi; ++b) {
      if (inv) inverse<L>(P, data + b * n, tmp.data());
      else forward<L>(P, data + b * n, tmp.data());
    }
  });
  return CR_OK;
}

template <int L>
int blas_t(int op, uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t n, const uint64_t* q,
           const uint64_t* alpha, uint32_t threads) {
  Mod<L> M;
  const int st = check_mod<L>(q, M);
  if (st != CR_OK) return st;
  if (op == OP_AXPY && (!alpha || geq<L>(alpha, M.q))) return CR_EINVAL;
  const Num<L>* pa = reinterpret_cast<const Num<L>*>(a);
  const Num<L>* pb = reinterpret_cast<const Num<L>*>(b);
  Num<L>* pc = reinterpret_cast<Num<L>*>(c);
  const uint64_t chunks = (n + 4095) / 4096;
  parallel(thread_count(threads, chunks), chunks, [&](uint64_t lo, uint64_t hi) {
    blas<L>(op, pc, pa, pb, lo * 4096, std::min(n, hi * 4096), M, alpha);
  });
  return CR_OK;
}

}  // namespace

extern "C" {

// Creates the tables of a transform of N = 2^log2n (1 <= log2n <= 17) points
// modulo q (`limbs` = 1, 2 or 4 words, q = 1 mod 2N, prime); psi is the
// primitive 2N-th root to use (limbs words) or NULL for the smallest one.
int cpuref_plan_create(void** plan, uint32_t log2n, const uint64_t* q, uint32_t limbs, const uint64_t* psi) {
  if (!plan || !q || log2n < 1 || log2n > 17) return CR_EINVAL;
  *plan = nullptr;
  PlanAny* A = nullptr;
  int st;
  if (limbs == 1) st = plan_create_t<1>(&A, log2n, q, psi);
  else if (limbs == 2) st = plan_create_t<2>(&A, log2n, q, psi);
  else if (limbs == 4) st = plan_create_t<4>(&A, log2n, q, psi);
  else return CR_EINVAL;
  if (st == CR_OK) *plan = A;
  return st;
}

// The plan's root psi (limbs words).
int cpuref_plan_root(void* plan, uint64_t* psi) {
  PlanAny* A = static_cast<PlanAny*>(plan);
  if (!A || !psi) return CR_EINVAL;
  // fwd[i] = psi^bitrev(i), so psi itself sits at index bitrev(1)
  if (A->limbs == 1) {
    const Plan<1>& P = *static_cast<Plan<1>*>(A->p);
    memcpy(psi, P.fwd[bitrev(1, P.log2n)].w, 8);
  } else if (A->limbs == 2) {
    const Plan<2>& P = *static_cast<Plan<2>*>(A->p);
    memcpy(psi, P.fwd[bitrev(1, P.log2n)].w, 16);
  } else {
    const Plan<4>& P = *static_cast<Plan<4>*>(A->p);
    memcpy(psi, P.fwd[bitrev(1, P.log2n)].w, 32);
  }
  return CR_OK;
}

int cpuref_plan_destroy(void* plan) {
  PlanAny* A = static_cast<PlanAny*>(plan);
  if (!A) return CR_EINVAL;
  if (A->limbs == 1) delete static_cast<Plan<1>*>(A->p);
  else if (A->limbs == 2) delete static_cast<Plan<2>*>(A->p);
  else delete static_cast<Plan<4>*>(A->p);
  delete A;
  return CR_OK;
}

// Forward (inverse = 0) or inverse transform of `batch` polynomials stored
// one after the other (N residues of `limbs` words each, canonical), natural
// order in and out; out may equal in.
int cpuref_ntt(void* plan, uint64_t* out, const uint64_t* in, uint32_t batch, uint32_t inverse, uint32_t threads) {
  PlanAny* A = static_cast<PlanAny*>(plan);
  if (!A || !out || !in) return CR_EINVAL;
  if (A->limbs == 1) return ntt_t<1>(A, out, in, batch, (int)inverse, threads);
  if (A->limbs == 2) return ntt_t<2>(A, out, in, batch, (int)inverse, threads);
  return ntt_t<4>(A, out, in, batch, (int)inverse, threads);
}

// c = a op b element-wise (op 0 add, 1 sub, 2 mul; 3 axpy: c = alpha*a + b),
// n residues of `limbs` words; c may equal a or b.
int cpuref_blas(uint32_t op, uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t n, const uint64_t* q,
                uint32_t limbs, const uint64_t* alpha, uint32_t threads) {
  if (!c || !a || !b || !q || op > OP_AXPY) return CR_EINVAL;
  if (n == 0) return CR_OK;
  if (limbs == 1) return blas_t<1>((int)op, c, a, b, n, q, alpha, threads);
  if (limbs == 2) return blas_t<2>((int)op, c, a, b, n, q, alpha, threads);
  if (limbs == 4) return blas_t<4>((int)op, c, a, b, n, q, alpha, threads);
  return CR_EINVAL;
}

}  // extern "C"
