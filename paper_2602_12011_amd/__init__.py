"""MI355X-native batched FP64 response generation and likelihood evaluation for
massive-black-hole-binary signals in LISA-, Taiji- and TianQin-like detectors
(arXiv:2602.12011).  The compute path is the C-ABI library ``libpes`` (HIP,
gfx950); this package holds its thin Python binding and the seeded workloads."""
