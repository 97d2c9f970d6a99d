// Host-side exact arithmetic for plan construction (moduli below 2^124).
//
// All values are unsigned __int128.  Products are reduced with a
// double-and-add loop (exact, no division instruction), and the precomputed
// constants of the device reductions come from bitwise long division:
//   shoup(w)   = floor(w * 2^(64L) / q)                     (Shoup companion)
//   barrett_mu = floor(2^(2T) / q'), q' = q * 2^(T - bitlen(q))  (Eq. barrett
//                on the modulus normalised to T = 60 or 124 bits)
// The canonical root of unity is the smallest primitive 2N-th root modulo q
// (the paper's Eq. (ntt) leaves the choice of root open).
#pragma once
#include <stdint.h>

namespace mwhost {

typedef unsigned __int128 u128;

inline int bitlen(u128 x) {
  int n = 0;
  while (x) { ++n; x >>= 1; }
  return n;
}

inline u128 addmod(u128 a, u128 b, u128 q) {  // a, b < q < 2^127
  u128 s = a + b;
  return s >= q ? s - q : s;
}

inline u128 submod(u128 a, u128 b, u128 q) { return a >= b ? a - b : a + (q - b); }

// a*b mod q by double-and-add over the bits of b (a, b < q < 2^126)
inline u128 mulmod(u128 a, u128 b, u128 q) {
  u128 r = 0;
  for (int i = bitlen(b) - 1; i >= 0; --i) {
    r = addmod(r, r, q);
    if ((b >> i) & 1) r = addmod(r, a, q);
  }
  return r;
}

inline u128 powmod(u128 a, u128 e, u128 q) {
  u128 r = 1 % q, base = a % q;
  while (e) {
    if (e & 1) r = mulmod(r, base, q);
    base = mulmod(base, base, q);
    e >>= 1;
  }
  return r;
}

// modular inverse for prime q (Fermat)
inline u128 invmod(u128 a, u128 q) { return powmod(a, q - 2, q); }

// floor(w * 2^shift / q) for w < q, shift <= 128 (result below 2^shift)
inline u128 shoup(u128 w, u128 q, int shift) {
  u128 quo = 0, rem = w;
  for (int i = 0; i < shift; ++i) {
    rem <<= 1;           // rem < q < 2^126, so no overflow
    quo <<= 1;
    if (rem >= q) { rem -= q; quo |= 1; }
  }
  return quo;
}

// floor(2^e / q) for q >= 1 below 2^124, e <= 2 * bitlen(q); result below 2^126
inline u128 pow2_div(int e, u128 q) {
  u128 quo = 0, rem = 0;
  for (int i = e; i >= 0; --i) {
    rem <<= 1;
    if (i == e) rem |= 1;  // the single set bit of 2^e
    quo <<= 1;
    if (rem >= q) { rem -= q; quo |= 1; }
  }
  return quo;
}

inline uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

// Smallest primitive 2N-th root of unity mod prime q (q = 1 mod 2N), or 0 if
// none is found.  psi0 = g^((q-1)/2N) for the first quadratic non-residue g has
// psi0^N = -1, and the primitive 2N-th roots are its odd powers.
inline u128 canonical_root(u128 q, uint32_t n) {
  if (q < 3 || !(q & 1) || ((q - 1) % (2 * (u128)n)) != 0) return 0;
  u128 g = 2;
  const u128 minus1 = q - 1;
  while (g < q && powmod(g, (q - 1) / 2, q) != minus1) ++g;
  if (g >= q) return 0;
  u128 psi0 = powmod(g, (q - 1) / (2 * (u128)n), q);
  if (powmod(psi0, n, q) != minus1) return 0;
  u128 sq = mulmod(psi0, psi0, q);
  u128 best = psi0, cur = psi0;
  for (uint32_t i = 1; i < n; ++i) {
    cur = mulmod(cur, sq, q);
    if (cur < best) best = cur;
  }
  return best;
}

inline u128 from_words(const uint64_t* w, uint32_t limbs) {
  u128 v = w[0];
  if (limbs > 1) v |= (u128)w[1] << 64;
  return v;
}

inline void to_words(u128 v, uint64_t* w, uint32_t limbs) {
  w[0] = (uint64_t)v;
  if (limbs > 1) w[1] = (uint64_t)(v >> 64);
}

}  // namespace mwhost
