// multislice.hip -- C ABI entry points adorym_forward / adorym_loss_grad and
// the context; the kernels live in multislice_impl.hpp and are
// instantiated per probe size and split in the ms_n*.hip units.
#include "multislice_impl.hpp"

using namespace adorym_ms;

extern template ADORYM_RUN_SIGNATURE(64, 4, 1);
extern template ADORYM_RUN_SIGNATURE(64, 4, 2);
extern template ADORYM_RUN_SIGNATURE(64, 4, 4);
extern template ADORYM_RUN_SIGNATURE(128, 8, 1);
extern template ADORYM_RUN_SIGNATURE(128, 8, 2);
extern template ADORYM_RUN_SIGNATURE(128, 8, 4);
extern template ADORYM_RUN_SIGNATURE(128, 8, 8);

namespace {

// Workgroups per position: the context's choice for this N if one was set
// (adorym_set_split, e.g. by an autotuner), else enough to cover the CUs.
int pick_split(const adorym_ctx* ctx, int n, int batch) {
  const int forced = n == 64 ? ctx->split64 : (n == 128 ? ctx->split128 : 0);
  if (forced > 0) return forced;
  // largest power-of-two split that keeps the grid within one workgroup per CU
  const int kmax = n == 64 ? 4 : 8;
  int k = 1;
  while (k < kmax && batch * (2 * k) <= 256) k *= 2;
  return k;
}

adorym_status dispatch(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                       const int32_t* corner, const float* shift, int batch, const float* i_meas, void* ws,
                       double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift, float* intensity,
                       bool with_loss) {
  const int k = pick_split(ctx, g->n, batch);
#define ADORYM_RUN(N_, L_, K_) \
  return run<N_, L_, K_>(ctx, g, a, b, probe, corner, shift, batch, i_meas, ws, loss, g_a, g_b, g_probe, g_shift, \
                         intensity, with_loss)
  if (g->n == 64) {
    switch (k) {
      case 1: ADORYM_RUN(64, 4, 1);
      case 2: ADORYM_RUN(64, 4, 2);
      case 4: ADORYM_RUN(64, 4, 4);
    }
  } else if (g->n == 128) {
    switch (k) {
      case 1: ADORYM_RUN(128, 8, 1);
      case 2: ADORYM_RUN(128, 8, 2);
      case 4: ADORYM_RUN(128, 8, 4);
      case 8: ADORYM_RUN(128, 8, 8);
    }
  }
#undef ADORYM_RUN
  return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size / split");
}

}  // namespace

extern "C" {

int adorym_supports_n(int32_t n) { return n == 64 || n == 128; }

adorym_status adorym_create(adorym_ctx** out, int device, void* stream) {
  if (!out) return ADORYM_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return ADORYM_EDEVICE;
  adorym_ctx* c = new adorym_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->msg[0] = 0;
  if (hipMalloc(&c->d_err, 256) != hipSuccess) { delete c; return ADORYM_EDEVICE; }
  if (hipMemset(c->d_err, 0, 256) != hipSuccess) { (void)hipFree(c->d_err); delete c; return ADORYM_EDEVICE; }
  *out = c;
  return ADORYM_OK;
}

adorym_status adorym_destroy(adorym_ctx* ctx) {
  if (!ctx) return ADORYM_EINVAL;
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  (void)hipFree(ctx->d_err);
  delete ctx;
  return ADORYM_OK;
}

adorym_status adorym_set_stream(adorym_ctx* ctx, void* stream) {
  if (!ctx) return ADORYM_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return ADORYM_OK;
}

size_t adorym_workspace_size(const adorym_geom* g, int32_t batch) {
  if (!g || batch < 1 || g->n < 1 || g->n_slices < 1 || g->ckpt_every < 1) return 0;
  return ws_layout(g, batch).total;
}

adorym_status adorym_forward(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                             const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                             float* intensity, void* workspace, size_t ws_bytes) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !intensity || !workspace)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (ws_bytes < adorym_workspace_size(g, batch)) return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  return dispatch(ctx, g, obj_a, obj_b, probe, corner, shift, batch, nullptr, workspace, nullptr, nullptr, nullptr,
                  nullptr, nullptr, intensity, false);
}

adorym_status adorym_loss_grad(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                               const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                               const float* i_meas, void* workspace, size_t ws_bytes, double* loss, float* g_a,
                               float* g_b, float* g_probe, float* g_shift, float* intensity) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !i_meas || !workspace || !loss)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if ((g_a == nullptr) != (g_b == nullptr)) return set_err(ctx, ADORYM_EINVAL, "g_a and g_b must both be given");
  if (ws_bytes < adorym_workspace_size(g, batch)) return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  return dispatch(ctx, g, obj_a, obj_b, probe, corner, shift, batch, i_meas, workspace, loss, g_a, g_b, g_probe,
                  g_shift, intensity, true);
}

adorym_status adorym_sync_error(adorym_ctx* ctx) {
  if (!ctx) return ADORYM_EINVAL;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, "stream sync failed");
  int flag = 0;
  if (hipMemcpy(&flag, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return set_err(ctx, ADORYM_EDEVICE, "reading the error flag failed");
  if (hipMemset(ctx->d_err, 0, sizeof(int)) != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, "clearing failed");
  if (flag & 2) return set_err(ctx, ADORYM_EDEVICE, "a workgroup group barrier timed out (groups not co-resident)");
  if (flag & 1) return set_err(ctx, ADORYM_ERANGE, "a chunk left the object; those positions contributed nothing");
  return ADORYM_OK;
}

const char* adorym_last_error_message(adorym_ctx* ctx) { return ctx ? ctx->msg : "no context"; }

adorym_status adorym_set_split(adorym_ctx* ctx, int32_t n, int32_t k) {
  if (!ctx) return ADORYM_EINVAL;
  const bool ok = k == 0 || (n == 64 && (k == 1 || k == 2 || k == 4)) ||
                  (n == 128 && (k == 1 || k == 2 || k == 4 || k == 8));
  if (!ok) return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size / split");
  if (n == 64) ctx->split64 = k;
  else ctx->split128 = k;
  return ADORYM_OK;
}

adorym_status adorym_profile_start(adorym_ctx* ctx, int32_t max_launches) {
  if (!ctx || max_launches < 1) return ADORYM_EINVAL;
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  ctx->ev.assign(2 * (size_t)max_launches, nullptr);
  for (auto& e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, "hipEventCreate failed");
  ctx->ev_used = 0;
  ctx->prof = true;
  return ADORYM_OK;
}

adorym_status adorym_profile_stop(adorym_ctx* ctx, double* total_ms, int32_t* launches) {
  if (!ctx || !total_ms || !launches) return ADORYM_EINVAL;
  ctx->prof = false;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, "stream sync failed");
  double tot = 0.0;
  for (int i = 0; i + 1 < ctx->ev_used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]) != hipSuccess)
      return set_err(ctx, ADORYM_EDEVICE, "hipEventElapsedTime failed");
    tot += ms;
  }
  *total_ms = tot;
  *launches = ctx->ev_used / 2;
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  ctx->ev.clear();
  ctx->ev_used = 0;
  return ADORYM_OK;
}

}  // extern "C"
