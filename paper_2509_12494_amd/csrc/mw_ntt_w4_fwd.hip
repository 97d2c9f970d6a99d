// NTT tile kernels: 4-word residues, fwd direction.
#define MW_W 4
#define MW_DIR 0
#include "mw_ntt_kernels.inc"
