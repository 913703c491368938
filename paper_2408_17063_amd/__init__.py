"""MI355X-native SIMD-aware homomorphic compression for private database queries.

The library is libhc.so (HIP for gfx950, C ABI in include/hc.h and
include/hc_kernels.h); `hc` is its Python binding. Build with
`paper_2408_17063_amd.build.build()`.
"""
