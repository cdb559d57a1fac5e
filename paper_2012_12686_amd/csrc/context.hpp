// context.hpp -- the library context behind the opaque adorym_ctx handle.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

struct adorym_ctx {
  int device;
  hipStream_t stream;
  int* d_err;          // deferred device error flags (bit 0: chunk out of range)
  char msg[512];
  // optional timing of the main multislice kernel (adorym_profile_*)
  std::vector<hipEvent_t> ev;   // start/stop pairs
  int ev_used = 0;
  bool prof = false;
  // workgroups per position (0 = automatic) for N = 64, 96, 128 and 192
  int split64 = 0, split96 = 0, split128 = 0, split192 = 0;
  // summed intensity of all probe modes [B][N][N] while adorym_loss_grad_modes
  // runs one mode's loss and gradient (the loss is taken at this intensity);
  // null otherwise
  const float* i_total = nullptr;
  // this device's copy of the static scratch array (adorym_forward_static),
  // as hipGetSymbolAddress returned it when the context was created
  void* scratch = nullptr;
};
