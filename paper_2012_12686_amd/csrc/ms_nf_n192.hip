// Kernel instantiations with near-field detector propagation: N=192 K=6.
#include "multislice_impl.hpp"

template ADORYM_RUN_NF_SIGNATURE(192, 16, 6);
