// Kernel instantiations: N=192 K=8.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(192, 16, 8);
template ADORYM_BATCHED_SIGNATURE(192, 16, 8);
