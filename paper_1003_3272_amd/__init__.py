"""MI355X-native multiplicative-update NMF: HIP kernels behind a C ABI
(include/nmf.h) with a thin ctypes binding (paper_1003_3272_amd.nmf)."""
