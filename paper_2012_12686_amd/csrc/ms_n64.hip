// Kernel instantiations: N=64 K=1, N=64 K=2, N=64 K=4 (8 lanes per line).
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(64, 8, 1);
template ADORYM_BATCHED_SIGNATURE(64, 8, 1);
template ADORYM_RUN_SIGNATURE(64, 8, 2);
template ADORYM_BATCHED_SIGNATURE(64, 8, 2);
template ADORYM_RUN_SIGNATURE(64, 8, 4);
template ADORYM_BATCHED_SIGNATURE(64, 8, 4);
template ADORYM_PARAMS_SIGNATURE(64, 4);
template ADORYM_PROLOGUE_SIGNATURE(64, 4);
template ADORYM_EPILOGUE_SIGNATURE(64, 4);
