// Kernel instantiations with unequal slice spacing: N=192 K=6.
#include "multislice_impl.hpp"

template ADORYM_RUN_GAPS_SIGNATURE(192, 16, 6);
