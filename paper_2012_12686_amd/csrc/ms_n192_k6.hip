// Kernel instantiations: N=192 K=6 (32 lines per workgroup: four waves, one per SIMD).
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(192, 8, 6);
template ADORYM_BATCHED_SIGNATURE(192, 8, 6);
