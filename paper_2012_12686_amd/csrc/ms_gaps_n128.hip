// Kernel instantiations with unequal slice spacing: N=128 K=4.
#include "multislice_impl.hpp"

template ADORYM_RUN_GAPS_SIGNATURE(128, 16, 4);
