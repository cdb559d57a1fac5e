// Kernel instantiations: N=128 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(128, 8, 1);
