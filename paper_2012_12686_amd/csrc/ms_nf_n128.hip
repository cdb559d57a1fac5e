// Kernel instantiations with near-field detector propagation: N=128 K=4.
#include "multislice_impl.hpp"

template ADORYM_RUN_NF_SIGNATURE(128, 16, 4);
