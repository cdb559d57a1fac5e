// Kernel instantiations of the deterministic mode (staged object gradients):
// N=64 and N=96, one workgroup per position.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(64, 4, 1, true);
template ADORYM_BATCHED_SIGNATURE(64, 4, 1, true);
template ADORYM_RUN_SIGNATURE(96, 8, 1, true);
template ADORYM_BATCHED_SIGNATURE(96, 8, 1, true);
