// Kernel instantiations: N=128 K=4.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(128, 8, 4);
template ADORYM_BATCHED_SIGNATURE(128, 8, 4);
