// Kernel instantiations with unequal slice spacing: N=96 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_GAPS_SIGNATURE(96, 8, 1);
