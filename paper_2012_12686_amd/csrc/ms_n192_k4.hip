// Kernel instantiations: N=192 K=4.
#include "multislice_impl.hpp"

template ADORYM_RUN_SIGNATURE(192, 8, 4);
template ADORYM_BATCHED_SIGNATURE(192, 8, 4);
template ADORYM_PARAMS_SIGNATURE(192, 8);
template ADORYM_PROLOGUE_SIGNATURE(192, 8);
template ADORYM_EPILOGUE_SIGNATURE(192, 8);
