// Host emulation of the device arithmetic (mw_arith.h, mw_butterfly.h) for
// the CPU pin test: the three CDNA instruction wrappers are replaced by exact
// host equivalents of their documented behaviour, everything else is the
// product's own code compiled for the host.
//
//   v_mad_u64_u32 d, c, a, b, acc : {c, d} = a * b + acc  (65-bit result)
//   v_addc_co_u32 d, -, x, 0, c   : d = x + (c's bit for this lane)
//   v_alignbit_b32 d, hi, lo, s   : d = ({hi, lo} >> (s & 31)) mod 2^32
//
// Reads one case per line from stdin and writes the result words in hex:
//   shoup  W q x w ws        -> T        (x < 2^(32W), w < q)
//   barrett W q a b          -> r
//   barrettk W q a b         -> r        (Barrett with the Karatsuba product)
//   kara W q a b             -> a*b      (2W words, any a, b < 2^(32W); q unused)
//   addmod / submod W q a b  -> r
//   ct     W q X Y w ws      -> X' Y'    (Cooley-Tukey, inputs in [0, 16q))
//   gs     W q X Y w ws      -> X' Y'    (Gentleman-Sande, inputs in [0, 8q))
//   gslast W q X Y n ns m ms -> X' Y'    (last inverse stage, N^-1 = n, m = w1 * N^-1)
//   canon  W q x             -> r        (x in [0, 16q))
// Every number is hexadecimal without prefix; W is 2, 4 or 8 32-bit words.
#include <stdint.h>

namespace mw {
inline uint64_t mad_cc(uint32_t a, uint32_t b, uint64_t& acc) {
  const unsigned __int128 t = (unsigned __int128)a * b + acc;
  acc = (uint64_t)t;
  return (uint64_t)(t >> 64);
}
inline uint32_t add_carry(uint32_t x, uint64_t cc) { return x + (uint32_t)(cc & 1u); }
inline uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (s & 31u));
}
}  // namespace mw

#define MW_ISA_EMULATED
#include "mw_butterfly.h"
#include "mw_common.h"

#include <cstdio>
#include <cstring>
#include <iostream>
#include <sstream>
#include <string>

using namespace mw;

namespace {

// hex string -> W little-endian 32-bit words (value must fit)
template <int W>
bool parse(const std::string& h, u32 (&out)[W]) {
  for (int i = 0; i < W; ++i) out[i] = 0;
  int bit = 0;
  for (int i = (int)h.size() - 1; i >= 0; --i) {
    const char c = h[i];
    const int v = c >= '0' && c <= '9' ? c - '0' : (c >= 'a' && c <= 'f' ? c - 'a' + 10 : -1);
    if (v < 0) return false;
    if (v && bit >= 32 * W) return false;
    if (bit < 32 * W) out[bit / 32] |= (u32)v << (bit % 32);
    bit += 4;
  }
  return true;
}

template <int W>
std::string hex(const u32 (&v)[W]) {
  std::string s;
  char buf[16];
  for (int i = W - 1; i >= 0; --i) {
    std::snprintf(buf, sizeof buf, "%08x", v[i]);
    s += buf;
  }
  return s;
}

template <int W>
Modulus<W> modulus(const u32 (&qw)[W]) {
  uint64_t q64[4] = {0, 0, 0, 0};
  for (int i = 0; i < W; ++i) q64[i / 2] |= (uint64_t)qw[i] << (32 * (i % 2));
  Modulus<W> M{};
  if constexpr (W == 8) make_modulus(q64, M);
  else make_modulus<W>(q64, W / 2, M);
  return M;
}

template <int W>
bool run(const std::string& op, std::istringstream& in, std::string& out) {
  std::string qs;
  in >> qs;
  u32 q[W];
  if (!parse<W>(qs, q)) return false;
  const Modulus<W> M = modulus<W>(q);
  std::string a1, a2, a3, a4, a5, a6;
  if (op == "shoup") {
    in >> a1 >> a2 >> a3;
    Res<W> x;
    u32 w[W], ws[W];
    if (!parse<W>(a1, x.v) || !parse<W>(a2, w) || !parse<W>(a3, ws)) return false;
    out = hex<W>(shoup_mul(x, w, ws, M).v);
  } else if (op == "kara") {
    in >> a1 >> a2;
    u32 a[W], b[W], r[2 * W];
    if (!parse<W>(a1, a) || !parse<W>(a2, b)) return false;
    mul_full_kara<W>(a, b, r);
    u32 hi[W], lo[W];
    for (int i = 0; i < W; ++i) {
      lo[i] = r[i];
      hi[i] = r[W + i];
    }
    out = hex<W>(hi) + hex<W>(lo);
  } else if (op == "barrettk") {
    in >> a1 >> a2;
    Res<W> a, b;
    if (!parse<W>(a1, a.v) || !parse<W>(a2, b.v)) return false;
    const Res<W> r = M.shift ? barrett_mul_t<W, true, true>(a, b, M) : barrett_mul_t<W, false, true>(a, b, M);
    out = hex<W>(r.v);
  } else if (op == "barrett" || op == "addmod" || op == "submod") {
    in >> a1 >> a2;
    Res<W> a, b;
    if (!parse<W>(a1, a.v) || !parse<W>(a2, b.v)) return false;
    const Res<W> r = op == "barrett" ? barrett_mul(a, b, M) : (op == "addmod" ? addmod(a, b, M) : submod(a, b, M));
    out = hex<W>(r.v);
  } else if (op == "ct" || op == "gs") {
    in >> a1 >> a2 >> a3 >> a4;
    Res<W> X, Y;
    Tw<W> t;
    if (!parse<W>(a1, X.v) || !parse<W>(a2, Y.v) || !parse<W>(a3, t.w) || !parse<W>(a4, t.ws)) return false;
    if (op == "ct") ct_bfly(X, Y, t, M);
    else gs_bfly(X, Y, t, M);
    out = hex<W>(X.v) + " " + hex<W>(Y.v);
  } else if (op == "gslast") {
    in >> a1 >> a2 >> a3 >> a4 >> a5 >> a6;
    Res<W> X, Y;
    Tw<W> n, m;
    if (!parse<W>(a1, X.v) || !parse<W>(a2, Y.v) || !parse<W>(a3, n.w) || !parse<W>(a4, n.ws) ||
        !parse<W>(a5, m.w) || !parse<W>(a6, m.ws))
      return false;
    gs_bfly_last(X, Y, n, m, M);
    out = hex<W>(X.v) + " " + hex<W>(Y.v);
  } else if (op == "canon") {
    in >> a1;
    Res<W> x;
    if (!parse<W>(a1, x.v)) return false;
    out = hex<W>(canon16(x, M).v);
  } else {
    return false;
  }
  return true;
}

}  // namespace

int main() {
  std::ios::sync_with_stdio(false);
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string op;
    int w = 0;
    in >> op >> w;
    std::string out;
    const bool ok = w == 2 ? run<2>(op, in, out) : (w == 4 ? run<4>(op, in, out) : (w == 8 && run<8>(op, in, out)));
    std::cout << (ok ? out : std::string("error")) << '\n';
  }
  return 0;
}
