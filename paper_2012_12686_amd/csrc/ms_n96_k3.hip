// Kernel instantiations: N=96 K=3 (16 lanes per line: eight waves, two per SIMD).
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(96, 16, 3);
template ADORYM_BATCHED_SIGNATURE(96, 16, 3);
