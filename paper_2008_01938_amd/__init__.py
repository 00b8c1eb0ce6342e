"""MI355X-native matrix-chain-multiplication DP solver (gfx950 HIP kernels)."""
