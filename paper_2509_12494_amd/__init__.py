"""Multi-word modular NTT and BLAS for MI355X (gfx950)."""
