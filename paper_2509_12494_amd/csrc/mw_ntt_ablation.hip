// Tile kernels of the arithmetic-variant plans (NTT_ARITH_MULHI /
// NTT_ARITH_CMPCARRY, the GPU analog of the paper's MQX ablation; the variant
// butterflies are in mw_ablation.h).  The variants run one shape: two-word
// transforms of 2^16 points as two passes of 2^8-point lines, 4 points per
// lane and 4 lines per 256-lane workgroup (the large-batch shape of the
// native plan at this size).
#include <hip/hip_runtime.h>

#include "mw_ablation.h"
#include "mw_ntt_tile.h"

#ifndef MWNTT_MIN_WAVES_PER_EU
#define MWNTT_MIN_WAVES_PER_EU 1
#endif

namespace mw {

constexpr u32 kVariantLogL = 8, kVariantLogP = 2, kVariantLines = 4;

template <int DIR, int MODE, class BF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MWNTT_MIN_WAVES_PER_EU)))
void ntt_variant_kernel(NttParams<4> p) {
  extern __shared__ __align__(16) unsigned char mw_smem[];
  const u32 tile = MODE == MODE_COL ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  ntt_tile<4, kVariantLogL, kVariantLogP, DIR, MODE, BF>(p, reinterpret_cast<Res<4>*>(mw_smem), tile);
}

template <class BF>
static hipError_t launch_variant(int dir, int mode, const NttParams<4>& p, u32 blocks, hipStream_t s) {
  if (p.lines != kVariantLines || (mode != MODE_COL && mode != MODE_ROW)) return hipErrorInvalidValue;
  const size_t lds = tile_lds_bytes<4>(kVariantLogL, kVariantLogP, kVariantLines);
  const dim3 threads(kVariantLines << (kVariantLogL - kVariantLogP));
  if (dir == DIR_FWD) {
    if (mode == MODE_COL)
      hipLaunchKernelGGL((ntt_variant_kernel<DIR_FWD, MODE_COL, BF>), dim3(blocks), threads, lds, s, p);
    else
      hipLaunchKernelGGL((ntt_variant_kernel<DIR_FWD, MODE_ROW, BF>), dim3(blocks), threads, lds, s, p);
  } else {
    if (mode == MODE_COL)
      hipLaunchKernelGGL((ntt_variant_kernel<DIR_INV, MODE_COL, BF>), dim3(blocks), threads, lds, s, p);
    else
      hipLaunchKernelGGL((ntt_variant_kernel<DIR_INV, MODE_ROW, BF>), dim3(blocks), threads, lds, s, p);
  }
  return hipGetLastError();
}

// variant: 1 multiply-high products, 2 compare-and-select carries, 3 both.
hipError_t launch_ntt_variant(int variant, int dir, int mode, const NttParams<4>& p, u32 blocks, hipStream_t s) {
  switch (variant) {
    case 1: return launch_variant<BflyVariant<IsaMulHi>>(dir, mode, p, blocks, s);
    case 2: return launch_variant<BflyVariant<IsaCmpCarry>>(dir, mode, p, blocks, s);
    case 3: return launch_variant<BflyVariant<IsaPlain>>(dir, mode, p, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mw
