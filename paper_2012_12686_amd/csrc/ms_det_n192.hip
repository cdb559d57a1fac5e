// Kernel instantiations of the deterministic mode (staged object gradients):
// N=192 split over 8 workgroups.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(192, 8, 8, true);
template ADORYM_BATCHED_SIGNATURE(192, 8, 8, true);
