// Kernel instantiations of the split evaluation (several probe modes): N=128 K=4.
#include "multislice_impl.hpp"

template ADORYM_RUN_SPLIT_SIGNATURE(128, 16, 4);
