// Kernel instantiations with unequal slice spacing: N=64 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_GAPS_SIGNATURE(64, 8, 1);
