// NTT tile kernels: 8-word residues, inv direction.
#define MW_W 8
#define MW_DIR 1
#include "mw_ntt_kernels.inc"
