// NTT tile kernels: 2-word residues, fwd direction.
#define MW_W 2
#define MW_DIR 0
#include "mw_ntt_kernels.inc"
