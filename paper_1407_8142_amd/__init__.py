"""MI355X (gfx950) levelwise wavelet-tree construction (Shun, "Parallel Wavelet Tree Construction").

The HIP library ``libwt.so`` does the work; ``wt`` binds it; ``inputs`` draws
seeded synthetic workloads.
"""
