// NTT tile kernels: 8-word residues, fwd direction.
#define MW_W 8
#define MW_DIR 0
#include "mw_ntt_kernels.inc"
