// Validate mode: canonicality checks of caller inputs (the paper's
// precondition 0 <= x < q of Eq. saddmod / ssubmod), see mw_set_validate in
// mwntt.h.  Internal interface for the entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mw {

// True while validate mode is on (first call reads MWNTT_VALIDATE).
bool validate_on();
// MW_ENONCANON if a check kernel has recorded a violation since the last
// report (the word is cleared), else MW_OK.  Does not synchronize.
int validate_take();
// Enqueues the check of `count` residues of `limbs` words at d_x against q on
// stream s (nothing when validate mode is off or count == 0).  MW_OK or
// MW_EDEVICE.
int validate_input(const void* d_x, uint64_t count, const uint64_t* q, uint32_t limbs, hipStream_t s);

}  // namespace mw
