"""MI355X-native kernel-polynomial (KPM/LSQT) density-of-states engine.

The compute path is the HIP library libtbkpm.so (C ABI declared in
include/tbkpm.h); `paper_2509_06525_amd.tbkpm` is its thin ctypes binding and
`paper_2509_06525_amd.synth` generates seeded synthetic inputs.
"""
