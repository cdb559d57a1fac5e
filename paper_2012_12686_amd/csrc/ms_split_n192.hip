// Kernel instantiations of the split evaluation (several probe modes): N=192 K=6.
#include "multislice_impl.hpp"

template ADORYM_RUN_SPLIT_SIGNATURE(192, 16, 6);
