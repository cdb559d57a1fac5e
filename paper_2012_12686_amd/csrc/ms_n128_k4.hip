// Kernel instantiations: N=128 K=4 (16 lanes per line: two waves per SIMD).
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(128, 16, 4);
template ADORYM_BATCHED_SIGNATURE(128, 16, 4);
