// NTT tile kernels: 2-word residues, inv direction.
#define MW_W 2
#define MW_DIR 1
#include "mw_ntt_kernels.inc"
