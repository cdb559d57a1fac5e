// Kernel instantiations: N=128 K=2.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(128, 8, 2);
template ADORYM_BATCHED_SIGNATURE(128, 8, 2);
