// Host stand-in for the few HIP declarations the arithmetic headers use, so
// that the CPU emulation test can compile them for the host (no device code).
#pragma once
#include <stdint.h>

#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))

struct uint2 {
  unsigned x, y;
};
struct uint4 {
  unsigned x, y, z, w;
};
inline uint2 make_uint2(unsigned x, unsigned y) { return uint2{x, y}; }
inline uint4 make_uint4(unsigned x, unsigned y, unsigned z, unsigned w) { return uint4{x, y, z, w}; }
