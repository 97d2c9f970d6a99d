// Host-side exact arithmetic for four-word moduli (q < 2^252): the plan and
// BLAS constants of the 256-bit path.
//
// Values are four little-endian 64-bit words.  Products of two residues are
// reduced with Barrett's method (Background, modular arithmetic, Eq. barrett)
// using the exact constant mu = floor(2^(2b) / q), b = bitlen(q), and full
// 512-bit products (no dropped columns), so at most two corrections follow.
// mu and the Shoup companions floor(w * 2^256 / q) come from bitwise long
// division, as in the 128-bit path.  The canonical root is found the same
// way as there: the smallest odd power of g^((q-1)/2N) for the first
// quadratic non-residue g.
#pragma once
#include <stdint.h>

namespace mwhost {

struct U256 {
  uint64_t w[4];
};

inline U256 u256(uint64_t lo) { return U256{{lo, 0, 0, 0}}; }

inline U256 u256_from_words(const uint64_t* x, uint32_t limbs) {
  U256 r = u256(0);
  for (uint32_t i = 0; i < limbs && i < 4; ++i) r.w[i] = x[i];
  return r;
}

inline void u256_to_words(const U256& v, uint64_t* x, uint32_t limbs) {
  for (uint32_t i = 0; i < limbs && i < 4; ++i) x[i] = v.w[i];
}

inline bool is_zero(const U256& a) { return !(a.w[0] | a.w[1] | a.w[2] | a.w[3]); }

// -1, 0, 1 as a <, ==, > b
inline int cmp(const U256& a, const U256& b) {
  for (int i = 3; i >= 0; --i) {
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  }
  return 0;
}

inline bool operator==(const U256& a, const U256& b) { return cmp(a, b) == 0; }
inline bool operator!=(const U256& a, const U256& b) { return cmp(a, b) != 0; }
inline bool operator<(const U256& a, const U256& b) { return cmp(a, b) < 0; }
inline bool operator>=(const U256& a, const U256& b) { return cmp(a, b) >= 0; }

// a + b mod 2^256; *carry (may be null) receives the carry out
inline U256 add(const U256& a, const U256& b, uint64_t* carry = nullptr) {
  U256 r;
  unsigned __int128 c = 0;
  for (int i = 0; i < 4; ++i) {
    c += (unsigned __int128)a.w[i] + b.w[i];
    r.w[i] = (uint64_t)c;
    c >>= 64;
  }
  if (carry) *carry = (uint64_t)c;
  return r;
}

// a - b mod 2^256
inline U256 sub(const U256& a, const U256& b) {
  U256 r;
  uint64_t borrow = 0;
  for (int i = 0; i < 4; ++i) {
    const uint64_t d = a.w[i] - b.w[i];
    const uint64_t b1 = a.w[i] < b.w[i];
    r.w[i] = d - borrow;
    borrow = b1 | (d < borrow);
  }
  return r;
}

inline U256 shl(const U256& a, int s) {  // 0 <= s < 64
  if (s == 0) return a;
  U256 r;
  for (int i = 3; i > 0; --i) r.w[i] = (a.w[i] << s) | (a.w[i - 1] >> (64 - s));
  r.w[0] = a.w[0] << s;
  return r;
}

inline U256 shl_any(U256 a, int s) {  // 0 <= s < 256, bits above 2^256 dropped
  while (s >= 64) {
    for (int i = 3; i > 0; --i) a.w[i] = a.w[i - 1];
    a.w[0] = 0;
    s -= 64;
  }
  return shl(a, s);
}

inline int bitlen(const U256& a) {
  for (int i = 3; i >= 0; --i) {
    if (a.w[i]) return 64 * i + 64 - __builtin_clzll(a.w[i]);
  }
  return 0;
}

inline bool bit(const U256& a, int i) { return (a.w[i >> 6] >> (i & 63)) & 1; }

// Full product a * b: 8 words.
inline void mul_wide(const U256& a, const U256& b, uint64_t (&out)[8]) {
  for (int i = 0; i < 8; ++i) out[i] = 0;
  for (int i = 0; i < 4; ++i) {
    unsigned __int128 c = 0;
    for (int j = 0; j < 4; ++j) {
      c += (unsigned __int128)a.w[i] * b.w[j] + out[i + j];
      out[i + j] = (uint64_t)c;
      c >>= 64;
    }
    out[i + 4] = (uint64_t)c;
  }
}

// Bits [s, s + 256) of an 8-word value, 0 <= s < 256.
inline U256 shr_window(const uint64_t (&x)[8], int s) {
  const int ws = s >> 6, bs = s & 63;
  U256 r;
  for (int i = 0; i < 4; ++i) {
    const uint64_t lo = x[ws + i];
    const uint64_t hi = (ws + i + 1 < 8) ? x[ws + i + 1] : 0;
    r.w[i] = bs ? (lo >> bs) | (hi << (64 - bs)) : lo;
  }
  return r;
}

// floor(2^e / q) for q >= 1, bitlen(q) <= 252, e <= 2 * bitlen(q); the
// quotient has at most e - bitlen(q) + 1 <= 253 bits.
inline U256 pow2_div(int e, const U256& q) {
  U256 quo = u256(0), rem = u256(0);
  for (int i = e; i >= 0; --i) {
    rem = shl(rem, 1);               // rem < q < 2^252: no overflow
    if (i == e) rem.w[0] |= 1;       // the single set bit of 2^e
    quo = shl(quo, 1);
    if (rem >= q) {
      rem = sub(rem, q);
      quo.w[0] |= 1;
    }
  }
  return quo;
}

// Shoup companion floor(w * 2^shift / q) for w < q < 2^252, shift <= 256
// (the quotient is below 2^shift).
inline U256 shoup(const U256& w, const U256& q, int shift) {
  U256 quo = u256(0), rem = w;
  for (int i = 0; i < shift; ++i) {
    rem = shl(rem, 1);
    quo = shl(quo, 1);
    if (rem >= q) {
      rem = sub(rem, q);
      quo.w[0] |= 1;
    }
  }
  return quo;
}

// A modulus with its Barrett constant.
struct Mod256 {
  U256 q, mu;
  int b;
};

inline Mod256 mod256(const U256& q) {
  Mod256 m;
  m.q = q;
  m.b = bitlen(q);
  m.mu = pow2_div(2 * m.b, q);
  return m;
}

// x mod q for x < q^2 (8 words), Barrett with exact products:
// q3 = floor(floor(x / 2^(b-1)) * mu / 2^(b+1)) is at most 2 below floor(x/q).
inline U256 reduce(const uint64_t (&x)[8], const Mod256& m) {
  const U256 q1 = shr_window(x, m.b - 1);   // < 2^(b+1)
  uint64_t q2[8];
  mul_wide(q1, m.mu, q2);
  const U256 q3 = shr_window(q2, m.b + 1);  // < 2^(b+1)
  uint64_t qq[8];
  mul_wide(q3, m.q, qq);
  // r = x - q3*q < 3q < 2^254: the low four words suffice
  U256 xl, ql;
  for (int i = 0; i < 4; ++i) {
    xl.w[i] = x[i];
    ql.w[i] = qq[i];
  }
  U256 r = sub(xl, ql);
  while (r >= m.q) r = sub(r, m.q);
  return r;
}

inline U256 mulmod(const U256& a, const U256& b, const Mod256& m) {
  uint64_t x[8];
  mul_wide(a, b, x);
  return reduce(x, m);
}

inline U256 powmod(const U256& a, const U256& e, const Mod256& m) {
  U256 r = u256(1), base = a;
  const int n = bitlen(e);
  for (int i = 0; i < n; ++i) {
    if (bit(e, i)) r = mulmod(r, base, m);
    base = mulmod(base, base, m);
  }
  return r;
}

// modular inverse for prime q (Fermat)
inline U256 invmod(const U256& a, const Mod256& m) { return powmod(a, sub(m.q, u256(2)), m); }

// (q - 1) / 2N for q = 1 mod 2N, N = 2^log2n
inline U256 exp_2n(const U256& q, uint32_t log2n) {
  U256 e = sub(q, u256(1));
  const int s = (int)log2n + 1;   // divide by 2^(log2n + 1) <= 2^18
  for (int i = 0; i < 4; ++i) {
    const uint64_t hi = (i + 1 < 4) ? e.w[i + 1] : 0;
    e.w[i] = (e.w[i] >> s) | (hi << (64 - s));
  }
  return e;
}

// q = 1 (mod 2^(log2n + 1))
inline bool one_mod_2n(const U256& q, uint32_t log2n) {
  const uint64_t mask = (uint64_t(2) << log2n) - 1;
  return (q.w[0] & mask) == 1;
}

// Smallest primitive 2N-th root of unity mod prime q, or zero if none is found.
inline U256 canonical_root(const Mod256& m, uint32_t log2n) {
  const U256& q = m.q;
  if (!(q.w[0] & 1) || bitlen(q) < 2 || !one_mod_2n(q, log2n)) return u256(0);
  const U256 minus1 = sub(q, u256(1));
  U256 half = minus1;   // (q - 1) / 2
  for (int i = 0; i < 4; ++i) half.w[i] = (half.w[i] >> 1) | (i + 1 < 4 ? half.w[i + 1] << 63 : 0);
  U256 g = u256(2);
  while (g < q && powmod(g, half, m) != minus1) g = add(g, u256(1));
  if (!(g < q)) return u256(0);
  const U256 psi0 = powmod(g, exp_2n(q, log2n), m);
  const uint32_t n = 1u << log2n;
  U256 nn = u256(n);
  if (powmod(psi0, nn, m) != minus1) return u256(0);
  const U256 sq = mulmod(psi0, psi0, m);
  U256 best = psi0, cur = psi0;
  for (uint32_t i = 1; i < n; ++i) {
    cur = mulmod(cur, sq, m);
    if (cur < best) best = cur;
  }
  return best;
}

}  // namespace mwhost
