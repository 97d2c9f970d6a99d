// NTT tile kernels: 4-word residues, inv direction.
#define MW_W 4
#define MW_DIR 1
#include "mw_ntt_kernels.inc"
