// Kernel instantiations of the split evaluation (several probe modes): N=64 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_SPLIT_SIGNATURE(64, 8, 1);
