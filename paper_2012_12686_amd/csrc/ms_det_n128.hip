// Kernel instantiations of the deterministic mode (staged object gradients):
// N=128 split over 4 workgroups.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(128, 8, 4, true);
template ADORYM_BATCHED_SIGNATURE(128, 8, 4, true);
