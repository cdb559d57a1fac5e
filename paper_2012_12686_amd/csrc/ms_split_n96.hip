// Kernel instantiations of the split evaluation (several probe modes): N=96 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_SPLIT_SIGNATURE(96, 8, 1);
