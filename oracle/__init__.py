"""Serial FP64 CPU oracle of the KPM density-of-states path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library.
"""
