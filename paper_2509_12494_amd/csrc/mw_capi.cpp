// C ABI: status strings and the host-only helpers (the plan's own arithmetic).
#include <stdint.h>

#include "../../include/mwntt.h"
#include "mw_host_math.h"
#include "mw_host_wide.h"

extern "C" const char* mw_status_str(int status) {
  switch (status) {
    case MW_OK: return "ok";
    case MW_EINVAL: return "invalid argument";
    case MW_EMODULUS: return "unsupported modulus";
    case MW_ESIZE: return "unsupported transform length";
    case MW_ENOMEM: return "out of memory";
    case MW_EDEVICE: return "HIP device error";
    case MW_EROOT: return "not a primitive 2N-th root of unity";
    case MW_EBUSY: return "request not complete";
    case MW_ENONCANON: return "input residue not canonical (validate mode)";
    default: return "unknown status";
  }
}

extern "C" const char* mw_version(void) { return "mwntt 0.1 (gfx950)"; }

static bool width_ok(mwhost::u128 q, uint32_t limbs) {
  if (limbs != 1 && limbs != 2) return false;
  int b = mwhost::bitlen(q);
  return (q & 1) && q >= 3 && b <= (limbs == 1 ? 60 : 124);
}

// four-word moduli: odd, 125 <= bitlen(q) <= 252
static bool wide_ok(const mwhost::U256& q) {
  const int b = mwhost::bitlen(q);
  return (q.w[0] & 1) && b >= 125 && b <= 252;
}

extern "C" int mw_canonical_root(const uint64_t* q, uint32_t limbs, uint32_t log2n, uint64_t* psi_out) {
  if (!q || !psi_out || (limbs != 1 && limbs != 2 && limbs != 4)) return MW_EINVAL;
  if (log2n < 1 || log2n > 17) return MW_ESIZE;
  if (limbs == 4) {
    const mwhost::U256 Q = mwhost::u256_from_words(q, 4);
    if (!wide_ok(Q) || !mwhost::one_mod_2n(Q, log2n)) return MW_EMODULUS;
    const mwhost::U256 r = mwhost::canonical_root(mwhost::mod256(Q), log2n);
    if (mwhost::is_zero(r)) return MW_EROOT;
    mwhost::u256_to_words(r, psi_out, 4);
    return MW_OK;
  }
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  if (!width_ok(Q, limbs)) return MW_EMODULUS;
  if ((Q - 1) % ((mwhost::u128)2 << log2n) != 0) return MW_EMODULUS;
  mwhost::u128 r = mwhost::canonical_root(Q, 1u << log2n);
  if (!r) return MW_EROOT;
  mwhost::to_words(r, psi_out, limbs);
  return MW_OK;
}

extern "C" int mw_shoup_companion(const uint64_t* w, const uint64_t* q, uint32_t limbs, uint64_t* out) {
  if (!w || !q || !out || (limbs != 1 && limbs != 2 && limbs != 4)) return MW_EINVAL;
  if (limbs == 4) {
    const mwhost::U256 Q = mwhost::u256_from_words(q, 4), Wv = mwhost::u256_from_words(w, 4);
    if (!wide_ok(Q)) return MW_EMODULUS;
    if (!(Wv < Q)) return MW_EINVAL;
    mwhost::u256_to_words(mwhost::shoup(Wv, Q, 256), out, 4);
    return MW_OK;
  }
  mwhost::u128 Q = mwhost::from_words(q, limbs), Wv = mwhost::from_words(w, limbs);
  if (!width_ok(Q, limbs)) return MW_EMODULUS;
  if (Wv >= Q) return MW_EINVAL;
  mwhost::to_words(mwhost::shoup(Wv, Q, 64 * (int)limbs), out, limbs);
  return MW_OK;
}

// Barrett constant of the normalised modulus: mu = floor(2^(2T) / q'),
// q' = q * 2^(T - bitlen(q)), T = 60, 124 or 252 for 1, 2 or 4 limbs.
extern "C" int mw_barrett_mu(const uint64_t* q, uint32_t limbs, uint64_t* out) {
  if (!q || !out || (limbs != 1 && limbs != 2 && limbs != 4)) return MW_EINVAL;
  if (limbs == 4) {
    const mwhost::U256 Q = mwhost::u256_from_words(q, 4);
    if (!wide_ok(Q)) return MW_EMODULUS;
    const mwhost::U256 Qn = mwhost::shl_any(Q, 252 - mwhost::bitlen(Q));
    mwhost::u256_to_words(mwhost::pow2_div(2 * 252, Qn), out, 4);
    return MW_OK;
  }
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  if (!width_ok(Q, limbs)) return MW_EMODULUS;
  const int T = limbs == 1 ? 60 : 124;
  mwhost::to_words(mwhost::pow2_div(2 * T, Q << (T - mwhost::bitlen(Q))), out, limbs);
  return MW_OK;
}
