// Kernel instantiations with near-field detector propagation: N=96 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_NF_SIGNATURE(96, 8, 1);
