// Kernel instantiations with near-field detector propagation: N=64 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_NF_SIGNATURE(64, 8, 1);
