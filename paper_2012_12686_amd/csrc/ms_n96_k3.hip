// Kernel instantiations: N=96 K=3 (32 lines per workgroup: four waves, one per SIMD).
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(96, 8, 3);
template ADORYM_BATCHED_SIGNATURE(96, 8, 3);
