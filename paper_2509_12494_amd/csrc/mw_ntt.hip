// Negacyclic NTT plans and entry points (host side).
//
// A plan holds, per (q, N): the forward table tw[i] = psi^bitrev(i) and the
// inverse table tw'[i] = psi^-bitrev(i), each entry with its Shoup companion
// floor(w * 2^(32W) / q), in device memory; N^-1 constants for the last
// inverse stage; the decomposition (single workgroup or N1 x N2 two-pass) and
// the tile shape of each pass; and a scratch buffer for the two-pass
// intermediate.  The transforms themselves are the tile kernels of
// mw_ntt_tile.h (see the algorithm notes there).
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <vector>

#include "mw_arith.h"
#include "mw_common.h"
#include "mw_exec.h"
#include "mw_ntt_tile.h"
#include "mw_tuned.h"
#include "mw_validate.h"

namespace mw {
// Arithmetic-variant tile kernels (mw_ntt_ablation.hip).
hipError_t launch_ntt_variant(int variant, int dir, int mode, const NttParams<4>& p, u32 blocks, hipStream_t s);

// Largest single-workgroup transform and points-per-lane exponent of a width
// (limbs 64-bit words per residue; see max_full_log / max_logp).
inline uint32_t max_full_for(uint32_t limbs) { return (uint32_t)max_full_log(2 * (int)limbs); }
inline uint32_t max_logp_for(uint32_t limbs) { return (uint32_t)max_logp(2 * (int)limbs); }
inline size_t tile_lds_for(uint32_t limbs, uint32_t logl, uint32_t logp, uint32_t lines) {
  return limbs == 4 ? tile_lds_bytes<8>(logl, logp, lines)
                    : (limbs == 2 ? tile_lds_bytes<4>(logl, logp, lines) : tile_lds_bytes<2>(logl, logp, lines));
}
}  // namespace mw

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
using namespace mw;

struct PassCfg {
  uint32_t logp = 3;          // points per lane, log2
  uint32_t lines = 8;         // lines per tile
};

struct PlanConfig {
  uint32_t log_n1 = 0;        // 0: single-workgroup transform
  PassCfg cfg[3];             // MODE_FULL, MODE_COL, MODE_ROW
};

struct ntt_plan_s {
  uint32_t log2n = 0, limbs = 0, flags = 0;
  // Two configurations: `lat` for calls with little work (one or a few
  // transforms: the shape that spreads one transform over the most CUs) and
  // `thr` for large batches.  A caller-set split / shape (`forced`) applies to
  // every call.
  PlanConfig lat, thr;
  bool forced = false;
  uint32_t variant = 0;       // arithmetic variant (NTT_ARITH_* flags), 0 native
  uint64_t q[4] = {0, 0, 0, 0};
  uint64_t psi[4] = {0, 0, 0, 0};
  int device = 0;
  void* d_tw_fwd = nullptr;   // N entries of {w, w'}
  void* d_tw_inv = nullptr;
  void* d_scratch = nullptr;  // two-pass intermediate
  uint32_t scratch_polys = 0;
  Modulus<8> M8;
  Modulus<4> M4;
  Modulus<2> M2;
  Tw<8> ninv8, last8;
  Tw<4> ninv4, last4;
  Tw<2> ninv2, last2;
};

namespace {

template <int W>
void fill_tw(Tw<W>& t, mwhost::u128 w, mwhost::u128 q) {
  put_words<W>(w, t.w);
  put_words<W>(mwhost::shoup(w, q, 32 * W), t.ws);
}

int upload_tables(ntt_plan_s* P, const void* fwd, const void* inv, size_t bytes);

template <int W>
int build_tables(ntt_plan_s* P, mwhost::u128 q, mwhost::u128 psi) {
  const uint32_t n = 1u << P->log2n;
  const int logn = (int)P->log2n;
  std::vector<Tw<W>> fwd(n), inv(n);
  mwhost::u128 psi_inv = mwhost::invmod(psi, q);
  // powers psi^e and psi^-e for e < N, then place at bit-reversed positions
  std::vector<mwhost::u128> pw(n), pwi(n);
  pw[0] = 1;
  pwi[0] = 1;
  for (uint32_t e = 1; e < n; ++e) {
    pw[e] = mwhost::mulmod(pw[e - 1], psi, q);
    pwi[e] = mwhost::mulmod(pwi[e - 1], psi_inv, q);
  }
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t e = mwhost::bitrev(i, logn);
    fill_tw<W>(fwd[i], pw[e], q);
    fill_tw<W>(inv[i], pwi[e], q);
  }
  mwhost::u128 ninv = mwhost::invmod((mwhost::u128)n, q);
  mwhost::u128 w1 = (n >= 2) ? pwi[mwhost::bitrev(1, logn)] : 1;
  Tw<W> tn, tl;
  fill_tw<W>(tn, ninv, q);
  fill_tw<W>(tl, mwhost::mulmod(w1, ninv, q), q);
  if constexpr (W == 4) {
    P->ninv4 = tn;
    P->last4 = tl;
  } else {
    P->ninv2 = tn;
    P->last2 = tl;
  }
  return upload_tables(P, fwd.data(), inv.data(), sizeof(Tw<W>) * n);
}

// Four-word moduli: the same tables from the 256-bit host arithmetic.
void fill_tw8(Tw<8>& t, const mwhost::U256& w, const mwhost::U256& q) {
  put_words<8>(w, t.w);
  put_words<8>(mwhost::shoup(w, q, 256), t.ws);
}

int upload_tables(ntt_plan_s* P, const void* fwd, const void* inv, size_t bytes) {
  if (hipMalloc(&P->d_tw_fwd, bytes) != hipSuccess) return MW_ENOMEM;
  if (hipMalloc(&P->d_tw_inv, bytes) != hipSuccess) return MW_ENOMEM;
  if (hipMemcpy(P->d_tw_fwd, fwd, bytes, hipMemcpyHostToDevice) != hipSuccess) return MW_EDEVICE;
  if (hipMemcpy(P->d_tw_inv, inv, bytes, hipMemcpyHostToDevice) != hipSuccess) return MW_EDEVICE;
  return MW_OK;
}

int build_tables8(ntt_plan_s* P, const mwhost::Mod256& m, const mwhost::U256& psi) {
  const uint32_t n = 1u << P->log2n;
  const int logn = (int)P->log2n;
  std::vector<Tw<8>> fwd(n), inv(n);
  const mwhost::U256 psi_inv = mwhost::invmod(psi, m);
  std::vector<mwhost::U256> pw(n), pwi(n);
  pw[0] = pwi[0] = mwhost::u256(1);
  for (uint32_t e = 1; e < n; ++e) {
    pw[e] = mwhost::mulmod(pw[e - 1], psi, m);
    pwi[e] = mwhost::mulmod(pwi[e - 1], psi_inv, m);
  }
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t e = mwhost::bitrev(i, logn);
    fill_tw8(fwd[i], pw[e], m.q);
    fill_tw8(inv[i], pwi[e], m.q);
  }
  const mwhost::U256 ninv = mwhost::invmod(mwhost::u256(n), m);
  const mwhost::U256 w1 = (n >= 2) ? pwi[mwhost::bitrev(1, logn)] : mwhost::u256(1);
  fill_tw8(P->ninv8, ninv, m.q);
  fill_tw8(P->last8, mwhost::mulmod(w1, ninv, m), m.q);
  return upload_tables(P, fwd.data(), inv.data(), sizeof(Tw<8>) * n);
}

void free_plan(ntt_plan_s* P) {
  if (!P) return;
  if (P->d_tw_fwd) (void)hipFree(P->d_tw_fwd);
  if (P->d_tw_inv) (void)hipFree(P->d_tw_inv);
  if (P->d_scratch) (void)hipFree(P->d_scratch);
  delete P;
}

// Scratch for the two-pass transforms.  A batch runs in chunks of as many
// polynomials as the scratch holds, two launches per chunk; each chunk
// boundary costs a few microseconds (measured: 2^16-point, 124-bit forward
// transforms take 1.70 us each in chunks of 64 and 1.51 us in one chunk of
// 256).  So the scratch holds 256 polynomials, within [64 MiB, 256 MiB] (and
// at least one polynomial).
constexpr size_t kScratchMin = size_t(64) << 20;
constexpr size_t kScratchMax = size_t(256) << 20;
constexpr size_t kScratchPolys = 256;

template <int W>
hipError_t launch_pass(int dir, int mode, const ntt_plan_s* P, const PlanConfig& C, NttParams<W>& p, u32 blocks,
                       hipStream_t s) {
  const u32 logl = mode == MODE_FULL ? P->log2n : (mode == MODE_COL ? C.log_n1 : P->log2n - C.log_n1);
  p.lines = C.cfg[mode].lines;
  if constexpr (W == 4) {
    if (P->variant) return launch_ntt_variant((int)P->variant, dir, mode, p, blocks, s);
  }
  return dir == DIR_FWD ? launch_ntt<W, DIR_FWD>(mode, logl, C.cfg[mode].logp, p, blocks, s)
                        : launch_ntt<W, DIR_INV>(mode, logl, C.cfg[mode].logp, p, blocks, s);
}

// Calls moving at least this many residues use the throughput configuration.
constexpr uint64_t kThroughputResidues = uint64_t(1) << 19;

const PlanConfig& pick_config(const ntt_plan_s* P, uint32_t batch) {
  if (P->forced) return P->lat;
  return ((uint64_t)batch << P->log2n) >= kThroughputResidues ? P->thr : P->lat;
}

// scratch / chunk: the two-pass intermediate and the polynomials it holds
// (the plan's own buffer, or the static one of ntt_transform_noalloc).
template <int W>
int run_transform(ntt_plan_s* P, void* d_out, const void* d_in, uint32_t batch, int dir, hipStream_t s,
                  void* scratch, uint32_t chunk) {
  NttParams<W> p = {};
  p.tw = reinterpret_cast<const Tw<W>*>(dir == DIR_FWD ? P->d_tw_fwd : P->d_tw_inv);
  if constexpr (W == 8) {
    p.M = P->M8;
    p.ninv = P->ninv8;
    p.ninv_w1 = P->last8;
  } else if constexpr (W == 4) {
    p.M = P->M4;
    p.ninv = P->ninv4;
    p.ninv_w1 = P->last4;
  } else {
    p.M = P->M2;
    p.ninv = P->ninv2;
    p.ninv_w1 = P->last2;
  }
  const PlanConfig& C = pick_config(P, batch);
  p.log_n = P->log2n;
  p.log_n1 = C.log_n1;
  const uint64_t N = 1ull << P->log2n;
  hipError_t e = hipSuccess;
  if (C.log_n1 == 0) {
    p.src = reinterpret_cast<const Res<W>*>(d_in);
    p.dst = reinterpret_cast<Res<W>*>(d_out);
    p.batch = batch;
    p.permute = dir == DIR_FWD ? !(P->flags & NTT_BITREV_OUT) : !(P->flags & NTT_BITREV_IN);
    const u32 lines = C.cfg[MODE_FULL].lines;
    e = launch_pass<W>(dir, MODE_FULL, P, C, p, (batch + lines - 1) / lines, s);
    return e == hipSuccess ? MW_OK : MW_EDEVICE;
  }
  const u32 col_tiles = tiles_per_poly<MODE_COL>(P->log2n, C.log_n1, C.cfg[MODE_COL].lines);
  const u32 row_tiles = tiles_per_poly<MODE_ROW>(P->log2n, C.log_n1, C.cfg[MODE_ROW].lines);
  for (uint32_t b0 = 0; b0 < batch; b0 += chunk) {
    const uint32_t nb = (batch - b0 < chunk) ? batch - b0 : chunk;
    const Res<W>* in = reinterpret_cast<const Res<W>*>(d_in) + (uint64_t)b0 * N;
    Res<W>* out = reinterpret_cast<Res<W>*>(d_out) + (uint64_t)b0 * N;
    Res<W>* scr = reinterpret_cast<Res<W>*>(scratch);
    p.batch = nb;
    if (dir == DIR_FWD) {
      p.src = in;
      p.dst = scr;
      p.permute = 0;
      e = launch_pass<W>(dir, MODE_COL, P, C, p, nb * col_tiles, s);
      if (e != hipSuccess) break;
      p.src = scr;
      p.dst = out;
      p.permute = !(P->flags & NTT_BITREV_OUT);
      e = launch_pass<W>(dir, MODE_ROW, P, C, p, nb * row_tiles, s);
    } else {
      p.src = in;
      p.dst = scr;
      p.permute = !(P->flags & NTT_BITREV_IN);
      e = launch_pass<W>(dir, MODE_ROW, P, C, p, nb * row_tiles, s);
      if (e != hipSuccess) break;
      p.src = scr;
      p.dst = out;
      p.permute = 0;
      e = launch_pass<W>(dir, MODE_COL, P, C, p, nb * col_tiles, s);
    }
    if (e != hipSuccess) break;
  }
  return e == hipSuccess ? MW_OK : MW_EDEVICE;
}

// Validate mode: report a pending violation, then check `batch` polynomials
// at d_in (see mw_set_validate).
int validate_polys(const ntt_plan_s* P, const void* d_in, uint32_t batch, hipStream_t s) {
  if (!validate_on()) return MW_OK;
  int st = validate_take();
  if (st != MW_OK) return st;
  return validate_input(d_in, (uint64_t)batch << P->log2n, P->q, P->limbs, s);
}

int transform(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream, int dir) {
  if (!plan) return MW_EINVAL;
  if (batch == 0) return MW_OK;
  if (!d_out || !d_in) return MW_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int vs = validate_polys(plan, d_in, batch, s);
  if (vs != MW_OK) return vs;
  switch (plan->limbs) {
    case 4: return run_transform<8>(plan, d_out, d_in, batch, dir, s, plan->d_scratch, plan->scratch_polys);
    case 2: return run_transform<4>(plan, d_out, d_in, batch, dir, s, plan->d_scratch, plan->scratch_polys);
    default: return run_transform<2>(plan, d_out, d_in, batch, dir, s, plan->d_scratch, plan->scratch_polys);
  }
}

// Default two-pass split: N1 = 2^floor(log N / 2) rows, N2 = N / N1.
uint32_t default_split(uint32_t log2n, uint32_t limbs) {
  if (log2n <= max_full_for(limbs)) return 0;
  return log2n / 2;
}

// Largest workgroup a tile kernel of this shape is compiled for (max_threads).
uint32_t thread_bound(uint32_t logl, uint32_t logp) {
  const uint32_t tpl = 1u << (logl - logp);
  return tpl > 256 ? (tpl > 1024 ? 1024 : tpl) : 256;
}

// Threads, LDS and shape limits of a tile configuration (see shape_ok).
bool tile_ok(uint32_t limbs, int mode, uint32_t logl, uint32_t logp, uint32_t lines, uint32_t max_lines) {
  if (logp < 1 || logp > max_logp_for(limbs) || logp > logl || logl - logp > 10) return false;
  if (mode == MODE_FULL) {
    if (logl < 1 || logl > max_full_for(limbs)) return false;
  } else if (logl < 3 || logl > 9) {
    return false;
  }
  if (lines == 0 || (lines & (lines - 1)) || lines > max_lines) return false;
  if (lines * (1u << (logl - logp)) > thread_bound(logl, logp)) return false;
  return tile_lds_for(limbs, logl, logp, lines) <= 160 * 1024;
}

// Default tile shapes: 8 points per lane (4 for four-word moduli); full
// tiles fill 256 lanes (or one line); column / row tiles take up to 8 lines
// (128-byte runs for two-word moduli) within the kernel's thread and LDS
// bounds.
void default_pass(PassCfg& c, uint32_t limbs, uint32_t logl, uint32_t max_lines) {
  const uint32_t lp_max = max_logp_for(limbs) < 3 ? max_logp_for(limbs) : 3;
  c.logp = logl < lp_max ? logl : lp_max;
  const uint32_t tpl = 1u << (logl - c.logp);
  uint32_t lines = 8;
  while (lines > 1 && (lines * tpl > thread_bound(logl, c.logp) || lines > max_lines ||
                       tile_lds_for(limbs, logl, c.logp, lines) > 160 * 1024))
    lines >>= 1;
  c.lines = lines;
}

void default_tiles(uint32_t logn, uint32_t limbs, PlanConfig& C) {
  const uint32_t lp_max = max_logp_for(limbs) < 3 ? max_logp_for(limbs) : 3;
  uint32_t lp = logn < lp_max ? logn : lp_max;
  uint32_t tpl = 1u << (logn - lp);
  while (tpl > 1024) { ++lp; tpl >>= 1; }
  C.cfg[MODE_FULL].logp = lp;
  C.cfg[MODE_FULL].lines = tpl >= 256 ? 1 : 256 / tpl;
  if (C.log_n1) {
    const uint32_t l1 = C.log_n1, l2 = logn - C.log_n1;
    default_pass(C.cfg[MODE_COL], limbs, l1, 1u << l2);
    default_pass(C.cfg[MODE_ROW], limbs, l2, 1u << l1);
  }
}

bool config_ok(uint32_t limbs, uint32_t logn, const PlanConfig& C) {
  if (C.log_n1 == 0) return tile_ok(limbs, MODE_FULL, logn, C.cfg[MODE_FULL].logp, C.cfg[MODE_FULL].lines, 1u << 16);
  const uint32_t l1 = C.log_n1, l2 = logn > l1 ? logn - l1 : 0;
  return tile_ok(limbs, MODE_COL, l1, C.cfg[MODE_COL].logp, C.cfg[MODE_COL].lines, 1u << l2) &&
         tile_ok(limbs, MODE_ROW, l2, C.cfg[MODE_ROW].logp, C.cfg[MODE_ROW].lines, 1u << l1);
}

// Default configurations, then the measured ones where the tuned table has
// an entry for this (width, N).
void initial_configs(ntt_plan_s* P) {
  P->lat.log_n1 = default_split(P->log2n, P->limbs);
  default_tiles(P->log2n, P->limbs, P->lat);
  P->thr = P->lat;
  for (const TunedCfg& t : kTuned) {
    if (t.limbs != P->limbs || t.log2n != P->log2n) continue;
    PlanConfig C;
    C.log_n1 = t.log_n1;
    C.cfg[MODE_FULL] = {t.full_logp, t.full_lines};
    C.cfg[MODE_COL] = {t.col_logp, t.col_lines};
    C.cfg[MODE_ROW] = {t.row_logp, t.row_lines};
    if (!config_ok(P->limbs, P->log2n, C)) continue;
    (t.kind == 0 ? P->lat : P->thr) = C;
  }
}

int ensure_scratch(ntt_plan_s* P) {
  if (P->d_scratch) return MW_OK;
  const size_t poly_bytes = (size_t)8 * P->limbs << P->log2n;
  size_t bytes = kScratchPolys * poly_bytes;
  bytes = bytes < kScratchMin ? kScratchMin : (bytes > kScratchMax ? kScratchMax : bytes);
  size_t polys = bytes / poly_bytes;
  if (polys < 1) polys = 1;
  if (hipMalloc(&P->d_scratch, polys * poly_bytes) != hipSuccess) return MW_ENOMEM;
  P->scratch_polys = (uint32_t)polys;
  return MW_OK;
}
}  // namespace

namespace mw {
// Read access to a plan for the batched executor (mw_exec.hip) and the
// serving runtime: the layout fields and the constants of its width.
bool plan_view(const ntt_plan_s* P, PlanView& v, ModConst<8>& c8, ModConst<4>& c4, ModConst<2>& c2) {
  if (!P) return false;
  v.log2n = P->log2n;
  v.limbs = P->limbs;
  v.flags = P->flags;
  v.variant = P->variant;
  v.q = P->q;
  v.tw_fwd = P->d_tw_fwd;
  v.tw_inv = P->d_tw_inv;
  if (P->limbs == 4) {
    c8.M = P->M8;
    c8.ninv = P->ninv8;
    c8.last = P->last8;
  } else if (P->limbs == 2) {
    c4.M = P->M4;
    c4.ninv = P->ninv4;
    c4.last = P->last4;
  } else {
    c2.M = P->M2;
    c2.ninv = P->ninv2;
    c2.last = P->last2;
  }
  return true;
}
}  // namespace mw

namespace {
// Host-only part of a plan: checks q = 1 (mod 2N), validates or finds the root
// (written to P->psi) and fills the per-modulus constants.  No device calls,
// so argument errors are reported without a device.
int setup_root(ntt_plan_s* P, const uint64_t* q, const uint64_t* psi) {
  const uint32_t limbs = P->limbs;
  const uint32_t n = 1u << P->log2n;
  if (limbs == 4) {
    const mwhost::U256 Q = mwhost::u256_from_words(q, 4);
    if (!mwhost::one_mod_2n(Q, P->log2n)) return MW_EMODULUS;
    const mwhost::Mod256 m = mwhost::mod256(Q);
    mwhost::U256 root;
    if (psi) {
      root = mwhost::u256_from_words(psi, 4);
      if (mwhost::is_zero(root) || !(root < Q) ||
          mwhost::powmod(root, mwhost::u256(n), m) != mwhost::sub(Q, mwhost::u256(1)))
        return MW_EROOT;
    } else {
      root = mwhost::canonical_root(m, P->log2n);
      if (mwhost::is_zero(root)) return MW_EROOT;
    }
    mwhost::u256_to_words(root, P->psi, 4);
    make_modulus(q, P->M8);
    return MW_OK;
  }
  mwhost::u128 Q = mwhost::from_words(q, limbs);
  if ((Q - 1) % (2 * (mwhost::u128)n) != 0) return MW_EMODULUS;
  mwhost::u128 root;
  if (psi) {
    root = mwhost::from_words(psi, limbs);
    if (root == 0 || root >= Q || mwhost::powmod(root, n, Q) != Q - 1) return MW_EROOT;
  } else {
    root = mwhost::canonical_root(Q, n);
    if (root == 0) return MW_EROOT;
  }
  mwhost::to_words(root, P->psi, limbs);
  if (limbs == 2) make_modulus<4>(q, limbs, P->M4);
  else make_modulus<2>(q, limbs, P->M2);
  return MW_OK;
}

// Device part: twiddle tables from P->q and P->psi.
int setup_tables(ntt_plan_s* P) {
  if (P->limbs == 4) {
    const mwhost::U256 Q = mwhost::u256_from_words(P->q, 4);
    return build_tables8(P, mwhost::mod256(Q), mwhost::u256_from_words(P->psi, 4));
  }
  const mwhost::u128 Q = mwhost::from_words(P->q, P->limbs), root = mwhost::from_words(P->psi, P->limbs);
  return P->limbs == 2 ? build_tables<4>(P, Q, root) : build_tables<2>(P, Q, root);
}
}  // namespace

extern "C" int ntt_plan(ntt_plan_t* out, uint32_t log2n, const uint64_t* q, uint32_t limbs,
                        const uint64_t* psi, uint32_t flags) {
  if (!out) return MW_EINVAL;
  *out = nullptr;
  if (flags & ~(NTT_BITREV_OUT | NTT_BITREV_IN | NTT_ARITH_MULHI | NTT_ARITH_CMPCARRY)) return MW_EINVAL;
  const uint32_t variant = (flags & NTT_ARITH_MULHI ? 1u : 0u) | (flags & NTT_ARITH_CMPCARRY ? 2u : 0u);
  if (variant && (limbs != 2 || log2n != 16)) return MW_EINVAL;
  if (log2n < 1 || log2n > 17) return MW_ESIZE;
  int st = check_modulus(q, limbs);
  if (st != MW_OK) return st;
  ntt_plan_s* P = new (std::nothrow) ntt_plan_s();
  if (!P) return MW_ENOMEM;
  P->log2n = log2n;
  P->limbs = limbs;
  P->flags = flags;
  for (uint32_t i = 0; i < limbs; ++i) P->q[i] = q[i];
  st = setup_root(P, q, psi);
  if (st == MW_OK && hipGetDevice(&P->device) != hipSuccess) st = MW_EDEVICE;
  if (st != MW_OK) {
    delete P;
    return st;
  }
  st = setup_tables(P);
  if (st != MW_OK) {
    free_plan(P);
    return st;
  }
  initial_configs(P);
  if (variant) {
    // the variant kernels' one shape, for every call
    P->variant = variant;
    P->forced = true;
    PlanConfig C;
    C.log_n1 = 8;
    C.cfg[MODE_COL] = {2, 4};
    C.cfg[MODE_ROW] = {2, 4};
    P->lat = P->thr = C;
  }
  if (P->lat.log_n1 || P->thr.log_n1) {
    st = ensure_scratch(P);
    if (st != MW_OK) {
      free_plan(P);
      return st;
    }
  }
  *out = P;
  return MW_OK;
}

namespace {
template <int W>
int run_pass(ntt_plan_s* P, uint32_t pass, void* d_out, const void* d_in, uint32_t batch, hipStream_t s) {
  const PlanConfig& C = pick_config(P, batch);
  if (C.log_n1 == 0) return MW_EINVAL;
  if (batch > P->scratch_polys) return MW_ESIZE;
  NttParams<W> p = {};
  p.tw = reinterpret_cast<const Tw<W>*>(P->d_tw_fwd);
  if constexpr (W == 8) {
    p.M = P->M8;
  } else if constexpr (W == 4) {
    p.M = P->M4;
  } else {
    p.M = P->M2;
  }
  p.log_n = P->log2n;
  p.log_n1 = C.log_n1;
  p.batch = batch;
  Res<W>* scr = reinterpret_cast<Res<W>*>(P->d_scratch);
  hipError_t e;
  if (pass == 1) {
    p.src = reinterpret_cast<const Res<W>*>(d_in);
    p.dst = scr;
    p.permute = 0;
    e = launch_pass<W>(DIR_FWD, MODE_COL, P, C, p,
                       batch * tiles_per_poly<MODE_COL>(P->log2n, C.log_n1, C.cfg[MODE_COL].lines), s);
  } else {
    p.src = scr;
    p.dst = reinterpret_cast<Res<W>*>(d_out);
    p.permute = !(P->flags & NTT_BITREV_OUT);
    e = launch_pass<W>(DIR_FWD, MODE_ROW, P, C, p,
                       batch * tiles_per_poly<MODE_ROW>(P->log2n, C.log_n1, C.cfg[MODE_ROW].lines), s);
  }
  return e == hipSuccess ? MW_OK : MW_EDEVICE;
}
}  // namespace

extern "C" int ntt_forward_pass(ntt_plan_t plan, uint32_t pass, void* d_out, const void* d_in, uint32_t batch,
                                void* stream) {
  if (!plan || (pass != 1 && pass != 2)) return MW_EINVAL;
  if (batch == 0) return MW_OK;
  if ((pass == 1 && !d_in) || (pass == 2 && !d_out)) return MW_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (validate_on()) {
    const int vs = pass == 1 ? validate_polys(plan, d_in, batch, s) : validate_take();
    if (vs != MW_OK) return vs;
  }
  switch (plan->limbs) {
    case 4: return run_pass<8>(plan, pass, d_out, d_in, batch, s);
    case 2: return run_pass<4>(plan, pass, d_out, d_in, batch, s);
    default: return run_pass<2>(plan, pass, d_out, d_in, batch, s);
  }
}

extern "C" int ntt_plan_set_split(ntt_plan_t plan, uint32_t log_n1) {
  if (!plan || plan->variant) return MW_EINVAL;
  const uint32_t max_full = max_full_for(plan->limbs);
  if (log_n1 == 0) {
    if (plan->log2n > max_full) return MW_ESIZE;
  } else {
    const uint32_t log_n2 = plan->log2n > log_n1 ? plan->log2n - log_n1 : 0;
    if (log_n1 < 3 || log_n1 > 9 || log_n2 < 3 || log_n2 > 9) return MW_ESIZE;
    int st = ensure_scratch(plan);
    if (st != MW_OK) return st;
  }
  plan->forced = true;
  plan->lat.log_n1 = log_n1;
  default_tiles(plan->log2n, plan->limbs, plan->lat);
  plan->thr = plan->lat;
  return MW_OK;
}

// The configuration a caller sees: the forced one, else the throughput one.
static PlanConfig& visible_config(ntt_plan_t plan) { return plan->forced ? plan->lat : plan->thr; }

extern "C" int ntt_plan_set_tiles(ntt_plan_t plan, uint32_t pass, uint32_t log_p, uint32_t lines) {
  if (!plan || pass > 2 || plan->variant) return MW_EINVAL;
  PlanConfig C = visible_config(plan);
  const uint32_t logn = plan->log2n;
  uint32_t logl, max_lines;
  if (pass == MODE_FULL) {
    if (C.log_n1) return MW_EINVAL;
    logl = logn;
    max_lines = 1u << 16;
  } else {
    if (!C.log_n1) return MW_EINVAL;
    logl = pass == MODE_COL ? C.log_n1 : logn - C.log_n1;
    max_lines = 1u << (pass == MODE_COL ? logn - C.log_n1 : C.log_n1);
  }
  if (!tile_ok(plan->limbs, (int)pass, logl, log_p, lines, max_lines)) return MW_EINVAL;
  if (C.log_n1) {
    int st = ensure_scratch(plan);
    if (st != MW_OK) return st;
  }
  C.cfg[pass].logp = log_p;
  C.cfg[pass].lines = lines;
  plan->forced = true;
  plan->lat = plan->thr = C;
  return MW_OK;
}

extern "C" int ntt_plan_get_tiles(ntt_plan_t plan, uint32_t pass, uint32_t* log_p, uint32_t* lines) {
  if (!plan || pass > 2 || !log_p || !lines) return MW_EINVAL;
  const PlanConfig& C = visible_config(plan);
  *log_p = C.cfg[pass].logp;
  *lines = C.cfg[pass].lines;
  return MW_OK;
}

extern "C" int ntt_plan_config_for(ntt_plan_t plan, uint32_t batch, uint32_t* large, uint32_t* log_n1) {
  if (!plan || !large || !log_n1) return MW_EINVAL;
  const PlanConfig& C = pick_config(plan, batch);
  *large = (!plan->forced && &C == &plan->thr) ? 1u : 0u;
  *log_n1 = C.log_n1;
  return MW_OK;
}

extern "C" int ntt_plan_get_split(ntt_plan_t plan, uint32_t* log_n1) {
  if (!plan || !log_n1) return MW_EINVAL;
  *log_n1 = visible_config(plan).log_n1;
  return MW_OK;
}

extern "C" int ntt_plan_destroy(ntt_plan_t plan) {
  if (!plan) return MW_EINVAL;
  (void)hipDeviceSynchronize();
  free_plan(plan);
  return MW_OK;
}

extern "C" int ntt_plan_root(ntt_plan_t plan, uint64_t* psi_out) {
  if (!plan || !psi_out) return MW_EINVAL;
  for (uint32_t i = 0; i < plan->limbs; ++i) psi_out[i] = plan->psi[i];
  return MW_OK;
}

extern "C" int ntt_forward(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream) {
  return transform(plan, d_out, d_in, batch, stream, DIR_FWD);
}

extern "C" int ntt_inverse(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream) {
  return transform(plan, d_out, d_in, batch, stream, DIR_INV);
}

// ---------------------------------------------------------------------------
// allocation-free transforms
// ---------------------------------------------------------------------------
// For callers that cannot allocate (code under stream capture, tight serving
// loops): the two-pass intermediate lives in a file-scope device array of
// kStaticScratchBytes that each device holds for the life of the process.  Its
// device address is looked up once per device (hipGetSymbolAddress with that
// device current) and only that address is used from host code; the symbol
// itself is not a device pointer on the host.  Every call on one device shares
// the array: calls that overlap in time on one device race.  Nothing in it
// needs clearing (the first pass writes every element the second reads).
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
int static_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MW_EDEVICE;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MW_EDEVICE;
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return MW_OK;
}
}  // namespace

extern "C" int ntt_transform_noalloc(ntt_plan_t plan, uint32_t inverse, void* d_out, const void* d_in,
                                     uint32_t batch, void* stream) {
  if (!plan || inverse > 1) return MW_EINVAL;
  if (batch == 0) return MW_OK;
  if (!d_out || !d_in) return MW_EINVAL;
  const int dir = inverse ? DIR_INV : DIR_FWD;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const PlanConfig& C = pick_config(plan, batch);
  void* scr = nullptr;
  uint32_t chunk = batch;
  if (C.log_n1) {
    const uint64_t need = ((uint64_t)batch * 8 * plan->limbs) << plan->log2n;
    if (need > kStaticScratchBytes) return MW_ESIZE;
    const int st = static_scratch(&scr);
    if (st != MW_OK) return st;
  }
  switch (plan->limbs) {
    case 4: return run_transform<8>(plan, d_out, d_in, batch, dir, s, scr, chunk);
    case 2: return run_transform<4>(plan, d_out, d_in, batch, dir, s, scr, chunk);
    default: return run_transform<2>(plan, d_out, d_in, batch, dir, s, scr, chunk);
  }
}
