// Kernel instantiations: N=128 K=8.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(128, 8, 8);
template ADORYM_BATCHED_SIGNATURE(128, 8, 8);
