// Kernel instantiations of the split evaluation (several probe modes; loss now,
// gradients later): N=128, K=4 and K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_SPLIT_SIGNATURE(128, 16, 4);
template ADORYM_RUN_SPLIT_SIGNATURE(128, 8, 1);
