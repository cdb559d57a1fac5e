// Kernel instantiations: N=192 K=6 (32 lines per workgroup, 16 lanes per line: eight waves, two per SIMD).
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(192, 16, 6);
template ADORYM_BATCHED_SIGNATURE(192, 16, 6);
