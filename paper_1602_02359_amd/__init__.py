"""MI355X-native hydrodynamics step of the FARGO3D method (arXiv:1602.02359).

`fargo` is the thin Python binding of the C-ABI library `libfargo.so`
(hand-written HIP kernels for gfx950); `workloads` builds seeded inputs.
"""
