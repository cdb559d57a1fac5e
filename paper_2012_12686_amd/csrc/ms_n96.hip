// Kernel instantiations: N=96 K=1, N=96 K=2, N=96 K=4.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(96, 8, 1);
template ADORYM_BATCHED_SIGNATURE(96, 8, 1);
template ADORYM_RUN_SIGNATURE(96, 8, 2);
template ADORYM_BATCHED_SIGNATURE(96, 8, 2);
template ADORYM_RUN_SIGNATURE(96, 8, 4);
template ADORYM_BATCHED_SIGNATURE(96, 8, 4);
template ADORYM_PARAMS_SIGNATURE(96, 8);
template ADORYM_PROLOGUE_SIGNATURE(96, 8);
template ADORYM_EPILOGUE_SIGNATURE(96, 8);
