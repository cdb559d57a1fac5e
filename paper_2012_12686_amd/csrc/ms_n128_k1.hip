// Kernel instantiations: N=128 K=1.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(128, 8, 1);
template ADORYM_BATCHED_SIGNATURE(128, 8, 1);
template ADORYM_PARAMS_SIGNATURE(128, 8);
template ADORYM_PROLOGUE_SIGNATURE(128, 8);
template ADORYM_EPILOGUE_SIGNATURE(128, 8);
