"""FP64 CPU oracle of the hydrodynamics step (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library.
"""
