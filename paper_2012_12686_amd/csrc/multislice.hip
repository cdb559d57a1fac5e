// multislice.hip -- C ABI entry points adorym_forward / adorym_loss_grad and
// the context; the kernels live in multislice_impl.hpp and are
// instantiated per probe size and split in the ms_n*.hip units.
#include "multislice_impl.hpp"

#include <mutex>

using namespace adorym_ms;

extern template ADORYM_RUN_SIGNATURE(64, 8, 1);
extern template ADORYM_BATCHED_SIGNATURE(64, 8, 1);
extern template ADORYM_RUN_SIGNATURE(64, 8, 2);
extern template ADORYM_BATCHED_SIGNATURE(64, 8, 2);
extern template ADORYM_RUN_SIGNATURE(64, 8, 4);
extern template ADORYM_BATCHED_SIGNATURE(64, 8, 4);
extern template ADORYM_RUN_SIGNATURE(96, 8, 1);
extern template ADORYM_BATCHED_SIGNATURE(96, 8, 1);
extern template ADORYM_RUN_SIGNATURE(96, 8, 2);
extern template ADORYM_BATCHED_SIGNATURE(96, 8, 2);
extern template ADORYM_RUN_SIGNATURE(96, 8, 4);
extern template ADORYM_BATCHED_SIGNATURE(96, 8, 4);
extern template ADORYM_RUN_SIGNATURE(128, 8, 1);
extern template ADORYM_BATCHED_SIGNATURE(128, 8, 1);
extern template ADORYM_RUN_SIGNATURE(128, 8, 2);
extern template ADORYM_BATCHED_SIGNATURE(128, 8, 2);
extern template ADORYM_RUN_SIGNATURE(128, 16, 4);
extern template ADORYM_BATCHED_SIGNATURE(128, 16, 4);
extern template ADORYM_RUN_SIGNATURE(128, 8, 8);
extern template ADORYM_BATCHED_SIGNATURE(128, 8, 8);
extern template ADORYM_RUN_SIGNATURE(192, 8, 2);
extern template ADORYM_BATCHED_SIGNATURE(192, 8, 2);
extern template ADORYM_RUN_SIGNATURE(192, 8, 4);
extern template ADORYM_BATCHED_SIGNATURE(192, 8, 4);
extern template ADORYM_RUN_SIGNATURE(192, 16, 6);
extern template ADORYM_BATCHED_SIGNATURE(192, 16, 6);
extern template ADORYM_RUN_SIGNATURE(96, 16, 3);
extern template ADORYM_BATCHED_SIGNATURE(96, 16, 3);
extern template ADORYM_RUN_SIGNATURE(192, 16, 8);
extern template ADORYM_BATCHED_SIGNATURE(192, 16, 8);
extern template ADORYM_RUN_SPLIT_SIGNATURE(64, 8, 1);
extern template ADORYM_RUN_SPLIT_SIGNATURE(96, 8, 1);
extern template ADORYM_RUN_SPLIT_SIGNATURE(128, 16, 4);
extern template ADORYM_RUN_SPLIT_SIGNATURE(128, 8, 1);
extern template ADORYM_RUN_SPLIT_SIGNATURE(192, 16, 6);
extern template ADORYM_RUN_NF_SIGNATURE(64, 8, 1);
extern template ADORYM_RUN_NF_SIGNATURE(96, 8, 1);
extern template ADORYM_RUN_NF_SIGNATURE(128, 16, 4);
extern template ADORYM_RUN_NF_SIGNATURE(192, 16, 6);
extern template ADORYM_RUN_GAPS_SIGNATURE(64, 8, 1);
extern template ADORYM_RUN_GAPS_SIGNATURE(96, 8, 1);
extern template ADORYM_RUN_GAPS_SIGNATURE(128, 16, 4);
extern template ADORYM_RUN_GAPS_SIGNATURE(192, 16, 6);
extern template ADORYM_PARAMS_SIGNATURE(64, 4);
extern template ADORYM_PROLOGUE_SIGNATURE(64, 4);
extern template ADORYM_EPILOGUE_SIGNATURE(64, 4);
extern template ADORYM_PARAMS_SIGNATURE(96, 8);
extern template ADORYM_PROLOGUE_SIGNATURE(96, 8);
extern template ADORYM_EPILOGUE_SIGNATURE(96, 8);
extern template ADORYM_PARAMS_SIGNATURE(128, 8);
extern template ADORYM_PROLOGUE_SIGNATURE(128, 8);
extern template ADORYM_EPILOGUE_SIGNATURE(128, 8);
extern template ADORYM_PARAMS_SIGNATURE(192, 8);
extern template ADORYM_PROLOGUE_SIGNATURE(192, 8);
extern template ADORYM_EPILOGUE_SIGNATURE(192, 8);

namespace {

int split_of(const adorym_ctx* ctx, int n) {
  switch (n) {
    case 64: return ctx->split64;
    case 96: return ctx->split96;
    case 128: return ctx->split128;
    case 192: return ctx->split192;
    default: return 0;
  }
}

// Workgroups per position: the context's choice for this N if one was set
// (adorym_set_split, e.g. by an autotuner), else enough to cover the CUs.
int pick_split(const adorym_ctx* ctx, int n, int batch) {
  const int forced = split_of(ctx, n);
  if (forced > 0) return forced;
  // N = 192: six workgroups of eight waves (two per SIMD)
  if (n == 192) return 6;
  // largest power-of-two split that keeps the grid within one workgroup per CU
  const int kmax = n == 128 ? 8 : 4;
  int k = 1;
  while (k < kmax && batch * (2 * k) <= 256) k *= 2;
  return k;
}

adorym_status dispatch(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                       const int32_t* corner, const float* shift, int batch, const float* i_meas, void* ws,
                       double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift, float* intensity,
                       bool with_loss, const Defocus* df = nullptr) {
  const int k = (g->flags & ADORYM_DETERMINISTIC) ? det_split(g->n) : pick_split(ctx, g->n, batch);
#define ADORYM_RUN(N_, L_, K_) \
  return run<N_, L_, K_>(ctx, g, a, b, probe, corner, shift, batch, i_meas, ws, loss, g_a, g_b, g_probe, g_shift, \
                         intensity, with_loss, df)
  if (g->n == 64) {
    switch (k) {
      case 1: ADORYM_RUN(64, 8, 1);
      case 2: ADORYM_RUN(64, 8, 2);
      case 4: ADORYM_RUN(64, 8, 4);
    }
  } else if (g->n == 96) {
    switch (k) {
      case 1: ADORYM_RUN(96, 8, 1);
      case 2: ADORYM_RUN(96, 8, 2);
      case 3: ADORYM_RUN(96, 16, 3);
      case 4: ADORYM_RUN(96, 8, 4);
    }
  } else if (g->n == 128) {
    switch (k) {
      case 1: ADORYM_RUN(128, 8, 1);
      case 2: ADORYM_RUN(128, 8, 2);
      case 4: ADORYM_RUN(128, 16, 4);
      case 8: ADORYM_RUN(128, 8, 8);
    }
  } else if (g->n == 192) {
    switch (k) {
      case 2: ADORYM_RUN(192, 8, 2);
      case 4: ADORYM_RUN(192, 8, 4);
      case 6: ADORYM_RUN(192, 16, 6);
      case 8: ADORYM_RUN(192, 16, 8);
    }
  }
#undef ADORYM_RUN
  return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size / split");
}

// Unequal slice spacing: one fixed split per probe size (that of the
// deterministic mode).
adorym_status dispatch_gaps(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b,
                            const float* probe, const int32_t* corner, const float* shift, int batch,
                            const double* gaps, const float* i_meas, void* ws, double* loss, float* g_a, float* g_b,
                            float* g_probe, float* g_shift, double* g_gaps, float* intensity, bool with_loss) {
#define ADORYM_RUN_GAPS(N_, L_, K_)                                                                              \
  return run_gaps<N_, L_, K_>(ctx, g, a, b, probe, corner, shift, batch, gaps, i_meas, ws, loss, g_a, g_b, g_probe, \
                              g_shift, g_gaps, intensity, with_loss)
  static_assert(det_split(64) == 1 && det_split(96) == 1 && det_split(128) == 4 && det_split(192) == 6,
                "unequal-spacing kernels are instantiated for the deterministic splits");
  switch (g->n) {
    case 64: ADORYM_RUN_GAPS(64, 8, 1);
    case 96: ADORYM_RUN_GAPS(96, 8, 1);
    case 128: ADORYM_RUN_GAPS(128, 16, 4);
    case 192: ADORYM_RUN_GAPS(192, 16, 6);
  }
#undef ADORYM_RUN_GAPS
  return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size");
}

// Near field: the same fixed splits.
adorym_status dispatch_nf(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                          const int32_t* corner, const float* shift, int batch, int kind, const double* dist,
                          int n_dist, const int32_t* idx, const float* i_meas, void* ws, double* loss, float* g_a,
                          float* g_b, float* g_probe, float* g_shift, double* g_dist, float* intensity,
                          bool with_loss) {
#define ADORYM_RUN_NF(N_, L_, K_)                                                                                    \
  return run_nf<N_, L_, K_>(ctx, g, a, b, probe, corner, shift, batch, kind, dist, n_dist, idx, i_meas, ws, loss, g_a, \
                            g_b, g_probe, g_shift, g_dist, intensity, with_loss)
  switch (g->n) {
    case 64: ADORYM_RUN_NF(64, 8, 1);
    case 96: ADORYM_RUN_NF(96, 8, 1);
    case 128: ADORYM_RUN_NF(128, 16, 4);
    case 192: ADORYM_RUN_NF(192, 16, 6);
  }
#undef ADORYM_RUN_NF
  return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size");
}


// ----------------------------------------------------------------------------
// Batched plans: many jobs of several probe sizes in persistent launches
// ----------------------------------------------------------------------------
struct PlanClass {
  int n, l, k, groups, repr;
  bool det;             // deterministic-mode jobs (fixed split)
  int n_items;
  int2* items;          // device [(job, position)] sorted by decreasing cost
  int* state;           // device: ticket, then mailbox[groups], counters[groups], xcc[groups*K]
  float2* xbuf;         // device [groups][4][N][N]
};

}  // namespace

struct adorym_plan {
  std::vector<adorym_job> jobs;
  std::vector<MsParams> params;     // host copy
  MsParams* d_params = nullptr;     // device job table
  std::vector<PlanClass> classes;
  std::vector<std::vector<int>> class_jobs;   // job indices of each class
  // Classes of one workgroup per position (K == 1) have no group barriers,
  // so they may share the chip: each runs on a stream of its own, forked
  // from the caller's stream and joined back (capturable in a HIP graph).
  std::vector<hipStream_t> side;    // one per K == 1 class, default priority
  std::vector<hipEvent_t> side_done;
  hipEvent_t fork = nullptr;
  int device = 0;
};

namespace {

template <int N, int L>
MsParams params_for(adorym_ctx* ctx, const adorym_job& j, int k) {
  MsParams P = make_params<N, L>(ctx, &j.g, j.obj_a, j.obj_b, j.batch, j.corner, j.shift, j.i_meas, j.workspace,
                                 j.g_probe != nullptr, j.g_a, j.g_b, j.intensity);
  P.ksplit = k;
  return P;
}

void job_prologue(const MsParams& P, const adorym_job& j, hipStream_t st) {
  switch (j.g.n) {
    case 64: launch_prologue<64, 4>(P, j.probe, &j.g, st, true); break;
    case 96: launch_prologue<96, 8>(P, j.probe, &j.g, st, true); break;
    case 128: launch_prologue<128, 8>(P, j.probe, &j.g, st, true); break;
    default: launch_prologue<192, 8>(P, j.probe, &j.g, st, true); break;
  }
}

void job_epilogue(const MsParams& P, const adorym_job& j, hipStream_t st) {
  switch (j.g.n) {
    case 64: launch_epilogue<64, 4>(P, j.workspace, &j.g, j.loss, j.g_probe, j.g_shift, st); break;
    case 96: launch_epilogue<96, 8>(P, j.workspace, &j.g, j.loss, j.g_probe, j.g_shift, st); break;
    case 128: launch_epilogue<128, 8>(P, j.workspace, &j.g, j.loss, j.g_probe, j.g_shift, st); break;
    default: launch_epilogue<192, 8>(P, j.workspace, &j.g, j.loss, j.g_probe, j.g_shift, st); break;
  }
}

void class_launch(const PlanClass& c, const MsParams* d_params, int* err, hipStream_t st) {
  const int n_state = 1 + 2 * c.groups + c.groups * c.k;
  hipLaunchKernelGGL(reset_ints_kernel, dim3((n_state + 255) / 256), dim3(256), 0, st, c.state, n_state);
  int* ticket = c.state;
  int* mailbox = c.state + 1;
  int* counters = mailbox + c.groups;
  int* xcc = counters + c.groups;
#define ADORYM_BATCH(N_, L_, K_) \
  launch_batched<N_, L_, K_>(d_params, c.items, c.n_items, ticket, mailbox, counters, xcc, c.xbuf, err, c.groups, \
                             c.repr, st)
  if (c.n == 64) {
    if (c.k == 1) ADORYM_BATCH(64, 8, 1); else if (c.k == 2) ADORYM_BATCH(64, 8, 2); else ADORYM_BATCH(64, 8, 4);
  } else if (c.n == 96) {
    if (c.k == 1) ADORYM_BATCH(96, 8, 1);
    else if (c.k == 2) ADORYM_BATCH(96, 8, 2);
    else if (c.k == 3) ADORYM_BATCH(96, 16, 3);
    else ADORYM_BATCH(96, 8, 4);
  } else if (c.n == 128) {
    if (c.k == 1) ADORYM_BATCH(128, 8, 1);
    else if (c.k == 2) ADORYM_BATCH(128, 8, 2);
    else if (c.k == 4) ADORYM_BATCH(128, 16, 4);
    else ADORYM_BATCH(128, 8, 8);
  } else {
    if (c.k == 2) ADORYM_BATCH(192, 8, 2);
    else if (c.k == 4) ADORYM_BATCH(192, 8, 4);
    else if (c.k == 6) ADORYM_BATCH(192, 16, 6);
    else ADORYM_BATCH(192, 16, 8);
  }
#undef ADORYM_BATCH
}

// dst += src (n floats); dst = 0 (n floats)
__global__ void add_into_kernel(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}
__global__ void zero_kernel(float* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = 0.f;
}

// Workspace of adorym_forward_static: a file-scope device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never
// uses its name as an address: each device's copy is looked up once with
// hipGetSymbolAddress (with that device current) and kept in
// g_scratch_addr.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The current device's scratch address, looked up on first use.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

int adorym_supports_n(int32_t n) { return n == 64 || n == 96 || n == 128 || n == 192; }

adorym_status adorym_create(adorym_ctx** out, int device, void* stream) {
  if (!out) return ADORYM_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return ADORYM_EDEVICE;
  adorym_ctx* c = new adorym_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->msg[0] = 0;
  if (scratch_address(device, &c->scratch) != hipSuccess) { delete c; return ADORYM_EDEVICE; }
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

size_t adorym_forward_workspace_size(const adorym_geom* g, int32_t batch) {
  if (!g || batch < 1 || g->n < 1 || g->n_slices < 1 || g->ckpt_every < 1) return 0;
  return ws_layout(g, batch, true).total;
}

adorym_status adorym_forward(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                             const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                             float* intensity, void* workspace, size_t ws_bytes) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !intensity || !workspace)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (ws_bytes < adorym_forward_workspace_size(g, batch))
    return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  return dispatch(ctx, g, obj_a, obj_b, probe, corner, shift, batch, nullptr, workspace, nullptr, nullptr, nullptr,
                  nullptr, nullptr, intensity, false);
}

adorym_status adorym_forward_static(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                                    const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                                    float* intensity) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !intensity)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  const size_t need = adorym_forward_workspace_size(g, batch);
  if (need > kStaticScratchBytes)
    return set_err(ctx, ADORYM_ENOMEM,
                   "forward workspace exceeds the 64 MiB static scratch: use adorym_forward with a workspace");
  if (!ctx->scratch) return set_err(ctx, ADORYM_EDEVICE, "no static scratch address on this device");
  return dispatch(ctx, g, obj_a, obj_b, probe, corner, shift, batch, nullptr, ctx->scratch, nullptr, nullptr,
                  nullptr, nullptr, nullptr, intensity, false);
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

// Probe defocus: the plain calls with the probe spectrum multiplied by the
// paraxial transfer function of the defocus distance (and, for the gradient,
// the chain rule back to the undefocused probe plus dL/d(defocus)).
static adorym_status make_defocus(adorym_ctx* ctx, const adorym_geom* g, double defocus_m, double* g_defocus,
                                  Defocus& df) {
  if (!std::isfinite(defocus_m)) return set_err(ctx, ADORYM_EINVAL, "defocus must be finite");
  df.dist = defocus_m;
  df.c0 = M_PI * g->wavelength_m / ((double)g->n * g->n * g->pixel_m * g->pixel_m);
  df.g_dist = g_defocus;
  return ADORYM_OK;
}

adorym_status adorym_forward_defocus(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                                     const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                                     double defocus_m, float* intensity, void* workspace, size_t ws_bytes) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !intensity || !workspace)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (ws_bytes < adorym_forward_workspace_size(g, batch))
    return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  Defocus df;
  st = make_defocus(ctx, g, defocus_m, nullptr, df);
  if (st != ADORYM_OK) return st;
  return dispatch(ctx, g, obj_a, obj_b, probe, corner, shift, batch, nullptr, workspace, nullptr, nullptr, nullptr,
                  nullptr, nullptr, intensity, false, &df);
}

adorym_status adorym_loss_grad_defocus(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a,
                                       const float* obj_b, const float* probe, const int32_t* corner,
                                       const float* shift, int32_t batch, double defocus_m, const float* i_meas,
                                       void* workspace, size_t ws_bytes, double* loss, float* g_a, float* g_b,
                                       float* g_probe, float* g_shift, double* g_defocus, float* intensity) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !i_meas || !workspace || !loss)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if ((g_a == nullptr) != (g_b == nullptr)) return set_err(ctx, ADORYM_EINVAL, "g_a and g_b must both be given");
  if (ws_bytes < adorym_workspace_size(g, batch)) return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  Defocus df;
  st = make_defocus(ctx, g, defocus_m, g_defocus, df);
  if (st != ADORYM_OK) return st;
  return dispatch(ctx, g, obj_a, obj_b, probe, corner, shift, batch, i_meas, workspace, loss, g_a, g_b, g_probe,
                  g_shift, intensity, true, &df);
}

// ---- Unequal slice spacing (sparse multislice) -----------------------------
size_t adorym_gaps_workspace_size(const adorym_geom* g, int32_t batch) {
  if (!g || batch < 1 || g->n < 1 || g->n_slices < 1 || g->ckpt_every < 1) return 0;
  return gaps_ws_size(g, batch, false);
}

adorym_status adorym_forward_gaps(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                                  const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                                  const double* gaps, float* intensity, void* workspace, size_t ws_bytes) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !intensity || !workspace)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (g->n_slices > 1 && !gaps) return set_err(ctx, ADORYM_EINVAL, "gaps is NULL");
  if (ws_bytes < adorym_forward_workspace_size(g, batch)) return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  return dispatch_gaps(ctx, g, obj_a, obj_b, probe, corner, shift, batch, gaps, nullptr, workspace, nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, intensity, false);
}

adorym_status adorym_loss_grad_gaps(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                                    const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                                    const double* gaps, const float* i_meas, void* workspace, size_t ws_bytes,
                                    double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift,
                                    double* g_gaps, float* intensity) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !i_meas || !workspace || !loss)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (g->n_slices > 1 && !gaps) return set_err(ctx, ADORYM_EINVAL, "gaps is NULL");
  if ((g_a == nullptr) != (g_b == nullptr)) return set_err(ctx, ADORYM_EINVAL, "g_a and g_b must both be given");
  if (ws_bytes < adorym_gaps_workspace_size(g, batch)) return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  return dispatch_gaps(ctx, g, obj_a, obj_b, probe, corner, shift, batch, gaps, i_meas, workspace, loss, g_a, g_b,
                       g_probe, g_shift, g_gaps, intensity, true);
}

// ---- Near field --------------------------------------------------------------
size_t adorym_nearfield_workspace_size(const adorym_geom* g, int32_t batch, int32_t n_dist) {
  if (!g || batch < 1 || g->n < 1 || g->n_slices < 1 || g->ckpt_every < 1 || n_dist < 1) return 0;
  return nf_layout(g, batch, n_dist).total;
}

static adorym_status check_nf(adorym_ctx* ctx, const adorym_geom* g, int batch, int kind, const double* dist,
                              int n_dist, const int32_t* idx, size_t ws_bytes) {
  if (kind != ADORYM_PROP_PARAXIAL && kind != ADORYM_PROP_SOMMERFELD)
    return set_err(ctx, ADORYM_EINVAL, "unknown near-field kernel");
  if (n_dist < 1 || !dist || !idx) return set_err(ctx, ADORYM_EINVAL, "distances and their indices are required");
  if (ws_bytes < adorym_nearfield_workspace_size(g, batch, n_dist))
    return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  return ADORYM_OK;
}

adorym_status adorym_forward_nearfield(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                                       const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                                       int32_t kind, const double* dist, int32_t n_dist, const int32_t* dist_idx,
                                       float* intensity, void* workspace, size_t ws_bytes) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !intensity || !workspace)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  st = check_nf(ctx, g, batch, kind, dist, n_dist, dist_idx, ws_bytes);
  if (st != ADORYM_OK) return st;
  return dispatch_nf(ctx, g, obj_a, obj_b, probe, corner, shift, batch, kind, dist, n_dist, dist_idx, nullptr,
                     workspace, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, intensity, false);
}

adorym_status adorym_loss_grad_nearfield(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a,
                                         const float* obj_b, const float* probe, const int32_t* corner,
                                         const float* shift, int32_t batch, int32_t kind, const double* dist,
                                         int32_t n_dist, const int32_t* dist_idx, const float* i_meas,
                                         void* workspace, size_t ws_bytes, double* loss, float* g_a, float* g_b,
                                         float* g_probe, float* g_shift, double* g_dist, float* intensity) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !i_meas || !workspace || !loss)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if ((g_a == nullptr) != (g_b == nullptr)) return set_err(ctx, ADORYM_EINVAL, "g_a and g_b must both be given");
  st = check_nf(ctx, g, batch, kind, dist, n_dist, dist_idx, ws_bytes);
  if (st != ADORYM_OK) return st;
  return dispatch_nf(ctx, g, obj_a, obj_b, probe, corner, shift, batch, kind, dist, n_dist, dist_idx, i_meas,
                     workspace, loss, g_a, g_b, g_probe, g_shift, g_dist, intensity, true);
}

// ---- Several incoherent probe modes --------------------------------------
// Workspace: a loss-and-gradient workspace, the summed and one mode's
// intensity, and per mode the checkpoints and the exit wave kept between
// the forward pass and the loss pass.
size_t adorym_modes_workspace_size(const adorym_geom* g, int32_t batch, int32_t n_modes) {
  const size_t one = adorym_workspace_size(g, batch);
  if (one == 0 || n_modes < 1) return 0;
  const size_t plane = align256((size_t)batch * g->n * g->n * sizeof(float));
  return one + 2 * plane + (size_t)n_modes * (split_ckpt_bytes(g, batch) + split_exit_bytes(g, batch));
}

adorym_status adorym_loss_grad_modes(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                                     const float* probes, int32_t n_modes, const int32_t* corner, const float* shift,
                                     int32_t batch, const float* i_meas, void* workspace, size_t ws_bytes,
                                     double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift,
                                     float* intensity) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (n_modes < 1) return set_err(ctx, ADORYM_EINVAL, "n_modes must be >= 1");
  if (!obj_a || !obj_b || !probes || !corner || !shift || !i_meas || !workspace || !loss)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if ((g_a == nullptr) != (g_b == nullptr)) return set_err(ctx, ADORYM_EINVAL, "g_a and g_b must both be given");
  if (ws_bytes < adorym_modes_workspace_size(g, batch, n_modes))
    return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  const size_t nn = (size_t)g->n * g->n, nb = (size_t)batch * nn;
  const size_t plane = align256(nb * sizeof(float));
  char* base = static_cast<char*>(workspace);
  void* ws = base;                                     // the loss-and-gradient workspace
  char* rest = base + adorym_workspace_size(g, batch);
  float* i_tot = reinterpret_cast<float*>(rest);
  float* i_mode = reinterpret_cast<float*>(rest + plane);
  char* per_mode = rest + 2 * plane;
  const size_t ck = split_ckpt_bytes(g, batch), ex = split_exit_bytes(g, batch);
  auto ckpt_of = [&](int m) { return reinterpret_cast<float2*>(per_mode + (size_t)m * (ck + ex)); };
  auto exit_of = [&](int m) { return reinterpret_cast<float2*>(per_mode + (size_t)m * (ck + ex) + ck); };
  hipStream_t s = ctx->stream;
  const int blocks = (int)std::min<size_t>((nb + 255) / 256, 4096);
  // one fixed split per probe size, as the deterministic mode
  auto pass = [&](const adorym_geom* gm, int m, bool with_loss, float* gp, float* inten) -> adorym_status {
    const float* pm = probes + (size_t)m * 2 * nn;
#define ADORYM_RUN_SPLIT(N_, L_, K_)                                                                               \
  return run_split<N_, L_, K_>(ctx, gm, obj_a, obj_b, pm, corner, shift, batch, with_loss ? i_meas : nullptr, ws, \
                               ckpt_of(m), exit_of(m), with_loss ? loss : nullptr, with_loss ? g_a : nullptr,      \
                               with_loss ? g_b : nullptr, gp, with_loss ? g_shift : nullptr, inten, with_loss, 1.0f)
    switch (g->n) {
      case 64: ADORYM_RUN_SPLIT(64, 8, 1);
      case 96: ADORYM_RUN_SPLIT(96, 8, 1);
      case 128: ADORYM_RUN_SPLIT(128, 16, 4);
      case 192: ADORYM_RUN_SPLIT(192, 16, 6);
    }
#undef ADORYM_RUN_SPLIT
    return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size");
  };
  // 1. every mode's forward pass: intensities summed, checkpoints and exit waves kept
  for (int m = 0; m < n_modes; ++m) {
    st = pass(g, m, false, nullptr, m == 0 ? i_tot : i_mode);
    if (st != ADORYM_OK) return st;
    if (m > 0) hipLaunchKernelGGL(add_into_kernel, dim3(blocks), dim3(256), 0, s, i_tot, i_mode, nb);
  }
  // 2. every mode's loss pass at the summed intensity; object and shift
  //    gradients add up over the modes, the probe gradient is per mode
  adorym_geom gm = *g;
  ctx->i_total = i_tot;
  for (int m = 0; m < n_modes && st == ADORYM_OK; ++m) {
    if (m > 0) gm.flags |= ADORYM_ACCUMULATE_GRADS;
    float* gp = g_probe ? g_probe + (size_t)m * 2 * nn : nullptr;
    if (gp && m > 0 && !(g->flags & ADORYM_ACCUMULATE_GRADS))
      hipLaunchKernelGGL(zero_kernel, dim3((int)std::min<size_t>((2 * nn + 255) / 256, 4096)), dim3(256), 0, s,
                         gp, 2 * nn);
    st = pass(&gm, m, true, gp, nullptr);
  }
  ctx->i_total = nullptr;
  if (st != ADORYM_OK) return st;
  if (intensity) (void)hipMemcpyAsync(intensity, i_tot, nb * sizeof(float), hipMemcpyDeviceToDevice, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return ADORYM_OK;
}

// ---- Loss first, gradients later -----------------------------------------
// Workspace: a loss-and-gradient workspace, the intensity plane, the
// checkpoints and exit waves kept between the calls, loss partials and a
// scratch loss.
namespace {
struct FwdLayout { size_t inten, ckpt, exit, part, scratch, total; };
FwdLayout fwd_layout(const adorym_geom* g, int batch) {
  FwdLayout l{};
  size_t off = adorym_workspace_size(g, batch);
  l.inten = off; off += align256((size_t)batch * g->n * g->n * sizeof(float));
  l.ckpt = off; off += split_ckpt_bytes(g, batch);
  l.exit = off; off += split_exit_bytes(g, batch);
  l.part = off; off += align256(kLossBlocks * sizeof(double));
  l.scratch = off; off += 256;
  l.total = off;
  return l;
}

// Split of loss-now / gradients-later: the deterministic split, except at
// N = 128 with more than 128 positions, where one workgroup per position
// already covers the CUs and the automatic rule of adorym_loss_grad picks
// K = 1 as well (the fixed K = 4 would be a quarter slower there).  It
// depends on N, the batch and the flags only, so adorym_loss_fwd and
// adorym_loss_bwd on the same arguments agree (the workspace's checkpoint and
// exit-wave slots are laid out per workgroup).
int split_pass_k(const adorym_geom* g, int batch) {
  if (g->n == 128 && !(g->flags & ADORYM_DETERMINISTIC) && 2 * batch > 256) return 1;
  return det_split(g->n);
}

adorym_status split_pass(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                         const int32_t* corner, const float* shift, int batch, const float* i_meas, void* ws,
                         float2* ckpt, float2* exit_wave, double* loss, float* g_a, float* g_b, float* g_probe,
                         float* g_shift, float* intensity, bool with_loss, float adj_scale) {
#define ADORYM_RUN_SPLIT(N_, L_, K_)                                                                                \
  return run_split<N_, L_, K_>(ctx, g, a, b, probe, corner, shift, batch, i_meas, ws, ckpt, exit_wave, loss, g_a, \
                               g_b, g_probe, g_shift, intensity, with_loss, adj_scale)
  switch (g->n) {
    case 64: ADORYM_RUN_SPLIT(64, 8, 1);
    case 96: ADORYM_RUN_SPLIT(96, 8, 1);
    case 128:
      if (split_pass_k(g, batch) == 1) ADORYM_RUN_SPLIT(128, 8, 1);
      ADORYM_RUN_SPLIT(128, 16, 4);
    case 192: ADORYM_RUN_SPLIT(192, 16, 6);
  }
#undef ADORYM_RUN_SPLIT
  return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size");
}
}  // namespace

size_t adorym_loss_fwd_workspace_size(const adorym_geom* g, int32_t batch) {
  if (adorym_workspace_size(g, batch) == 0) return 0;
  return fwd_layout(g, batch).total;
}

adorym_status adorym_loss_fwd(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                              const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                              const float* i_meas, void* workspace, size_t ws_bytes, double* loss,
                              float* intensity) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !i_meas || !workspace || !loss)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (ws_bytes < adorym_loss_fwd_workspace_size(g, batch)) return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  const FwdLayout l = fwd_layout(g, batch);
  char* base = static_cast<char*>(workspace);
  float* inten = reinterpret_cast<float*>(base + l.inten);
  st = split_pass(ctx, g, obj_a, obj_b, probe, corner, shift, batch, nullptr, workspace,
                  reinterpret_cast<float2*>(base + l.ckpt), reinterpret_cast<float2*>(base + l.exit), nullptr, nullptr,
                  nullptr, nullptr, nullptr, inten, false, 1.0f);
  if (st != ADORYM_OK) return st;
  const size_t n = (size_t)batch * g->n * g->n;
  double* part = reinterpret_cast<double*>(base + l.part);
  hipLaunchKernelGGL(loss_value_kernel, dim3(kLossBlocks), dim3(256), 0, ctx->stream, inten, i_meas, n, g->loss,
                     (float)g->eps, part);
  hipLaunchKernelGGL(finish_loss_kernel, dim3(1), dim3(256), 0, ctx->stream, part, 1.0 / (double)n, loss);
  if (intensity) (void)hipMemcpyAsync(intensity, inten, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return ADORYM_OK;
}

adorym_status adorym_loss_bwd(adorym_ctx* ctx, const adorym_geom* g, const float* obj_a, const float* obj_b,
                              const float* probe, const int32_t* corner, const float* shift, int32_t batch,
                              const float* i_meas, void* workspace, size_t ws_bytes, double grad_scale, float* g_a,
                              float* g_b, float* g_probe, float* g_shift) {
  adorym_status st = check_geom(ctx, g, batch);
  if (st != ADORYM_OK) return st;
  if (!obj_a || !obj_b || !probe || !corner || !shift || !i_meas || !workspace)
    return set_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if ((g_a == nullptr) != (g_b == nullptr)) return set_err(ctx, ADORYM_EINVAL, "g_a and g_b must both be given");
  if (!(grad_scale == grad_scale) || grad_scale > 3.0e38 || grad_scale < -3.0e38)
    return set_err(ctx, ADORYM_EINVAL, "grad_scale must be a finite float32 value");
  if (ws_bytes < adorym_loss_fwd_workspace_size(g, batch)) return set_err(ctx, ADORYM_ENOMEM, "workspace too small");
  const FwdLayout l = fwd_layout(g, batch);
  char* base = static_cast<char*>(workspace);
  return split_pass(ctx, g, obj_a, obj_b, probe, corner, shift, batch, i_meas, workspace,
                    reinterpret_cast<float2*>(base + l.ckpt), reinterpret_cast<float2*>(base + l.exit),
                    reinterpret_cast<double*>(base + l.scratch), g_a, g_b, g_probe, g_shift, nullptr, true,
                    (float)grad_scale);
}

// ---- Many jobs in one call ---------------------------------------------------
adorym_status adorym_loss_grad_batched(adorym_ctx* ctx, const adorym_job* jobs, int32_t n_jobs) {
  adorym_plan* plan = nullptr;
  adorym_status st = adorym_plan_create(ctx, jobs, n_jobs, &plan);
  if (st != ADORYM_OK) return st;
  st = adorym_plan_run(ctx, plan);
  const hipError_t e = hipStreamSynchronize(ctx->stream);     // the plan's tables are freed next
  const adorym_status st2 = adorym_plan_destroy(plan);
  if (st != ADORYM_OK) return st;
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return st2;
}

// ---- Split per probe size from timed plan runs ------------------------------
adorym_status adorym_autotune(adorym_ctx* ctx, const adorym_job* jobs, int32_t n_jobs, int32_t reps,
                              int32_t* chosen) {
  if (!ctx) return ADORYM_EINVAL;
  if (!jobs || n_jobs < 1 || reps < 1) return set_err(ctx, ADORYM_EINVAL, "jobs and reps >= 1 are required");
  static const int kSizes[4] = {64, 96, 128, 192};
  static const int kCand[4][4] = {{1, 2, 4, 0}, {1, 2, 3, 4}, {1, 2, 4, 8}, {2, 4, 6, 8}};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, "event creation failed");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return set_err(ctx, ADORYM_EDEVICE, "event creation failed"); }
  adorym_status st = ADORYM_OK;
  for (int si = 0; si < 4 && st == ADORYM_OK; ++si) {
    const int n = kSizes[si];
    std::vector<adorym_job> sub;
    for (int i = 0; i < n_jobs; ++i)
      if (jobs[i].g.n == n && !(jobs[i].g.flags & ADORYM_DETERMINISTIC)) sub.push_back(jobs[i]);
    if (sub.empty()) {
      if (chosen) chosen[si] = split_of(ctx, n);
      continue;
    }
    int best = 0;
    float best_ms = 0.f;
    for (int c = 0; c < 4 && st == ADORYM_OK; ++c) {
      const int k = kCand[si][c];
      if (k == 0) continue;
      st = adorym_set_split(ctx, n, k);
      adorym_plan* plan = nullptr;
      if (st == ADORYM_OK) st = adorym_plan_create(ctx, sub.data(), (int32_t)sub.size(), &plan);
      if (st != ADORYM_OK) break;
      st = adorym_plan_run(ctx, plan);                     // warm-up
      (void)hipEventRecord(e0, ctx->stream);
      for (int r = 0; r < reps && st == ADORYM_OK; ++r) st = adorym_plan_run(ctx, plan);
      (void)hipEventRecord(e1, ctx->stream);
      float ms = 0.f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = set_err(ctx, ADORYM_EDEVICE, "timing failed");
      (void)adorym_plan_destroy(plan);
      if (st == ADORYM_OK && (best == 0 || ms < best_ms)) { best = k; best_ms = ms; }
    }
    if (st == ADORYM_OK) {
      st = adorym_set_split(ctx, n, best);
      if (chosen) chosen[si] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

adorym_status adorym_sync_error(adorym_ctx* ctx) {
  if (!ctx) return ADORYM_EINVAL;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, "stream sync failed");
  int flag = 0;
  if (hipMemcpy(&flag, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return set_err(ctx, ADORYM_EDEVICE, "reading the error flag failed");
  if (hipMemset(ctx->d_err, 0, sizeof(int)) != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, "clearing failed");
  if (flag & 2) return set_err(ctx, ADORYM_EDEVICE, "a workgroup group barrier timed out (groups not co-resident)");
  if (flag & 4) return set_err(ctx, ADORYM_EINVAL, "a distance index was outside the distance list; those positions contributed nothing");
  if (flag & 8) return set_err(ctx, ADORYM_EINVAL, "an Adam step read an iteration count below 1; it changed nothing");
  if (flag & 1) return set_err(ctx, ADORYM_ERANGE, "a chunk left the object; those positions contributed nothing");
  return ADORYM_OK;
}

const char* adorym_last_error_message(adorym_ctx* ctx) { return ctx ? ctx->msg : "no context"; }

adorym_status adorym_plan_create(adorym_ctx* ctx, const adorym_job* jobs, int32_t n_jobs, adorym_plan** out) {
  if (!ctx || !jobs || !out || n_jobs < 1) return ADORYM_EINVAL;
  *out = nullptr;
  adorym_plan* plan = new adorym_plan();
  plan->device = ctx->device;
  plan->jobs.assign(jobs, jobs + n_jobs);
  // validate every job; the plan's kernels are the loss+gradient path
  for (int i = 0; i < n_jobs; ++i) {
    const adorym_job& j = jobs[i];
    adorym_status st = check_geom(ctx, &j.g, j.batch);
    if (st == ADORYM_OK && (!j.obj_a || !j.obj_b || !j.probe || !j.corner || !j.shift || !j.i_meas || !j.workspace ||
                            !j.loss))
      st = set_err(ctx, ADORYM_EINVAL, "NULL array argument in a job");
    if (st == ADORYM_OK && ((j.g_a == nullptr) != (j.g_b == nullptr)))
      st = set_err(ctx, ADORYM_EINVAL, "g_a and g_b must both be given");
    if (st == ADORYM_OK && j.ws_bytes < adorym_workspace_size(&j.g, j.batch))
      st = set_err(ctx, ADORYM_ENOMEM, "job workspace too small");
    if (st != ADORYM_OK) { delete plan; return st; }
  }
  // classes: one per (probe size, object representation, deterministic mode)
  struct Key { int n, repr; bool det; };
  auto key_of = [](const adorym_job& j) {
    return Key{j.g.n, j.g.obj_repr, (j.g.flags & ADORYM_DETERMINISTIC) != 0};
  };
  auto same = [](const Key& x, const Key& y) { return x.n == y.n && x.repr == y.repr && x.det == y.det; };
  std::vector<Key> keys;
  for (const adorym_job& j : plan->jobs) {
    bool seen = false;
    for (const Key& k : keys) seen |= same(k, key_of(j));
    if (!seen) keys.push_back(key_of(j));
  }
  plan->params.resize(n_jobs);
  for (const Key& key : keys) {
    PlanClass c{};
    c.n = key.n; c.repr = key.repr; c.det = key.det;
    c.l = key.n == 64 ? 4 : 8;
    int class_items = 0;
    for (const adorym_job& j : plan->jobs)
      if (same(key_of(j), key)) class_items += j.batch;
    // the context's split if one was set, else the single-call rule applied
    // to all positions of the class
    c.k = c.det ? det_split(key.n) : pick_split(ctx, key.n, class_items);
    // one workgroup per CU: 256 / K groups, a multiple of 8 (one per XCD slot)
    c.groups = std::max(8, (256 / c.k) / 8 * 8);
    std::vector<std::pair<double, int2>> work;
    for (int i = 0; i < n_jobs; ++i) {
      const adorym_job& j = plan->jobs[i];
      if (!same(key_of(j), key)) continue;
      switch (key.n) {
        case 64: plan->params[i] = params_for<64, 4>(ctx, j, c.k); break;
        case 96: plan->params[i] = params_for<96, 8>(ctx, j, c.k); break;
        case 128: plan->params[i] = params_for<128, 8>(ctx, j, c.k); break;
        default: plan->params[i] = params_for<192, 8>(ctx, j, c.k); break;
      }
      for (int b = 0; b < j.batch; ++b) work.push_back({(double)j.g.n_slices * j.g.n * j.g.n, make_int2(i, b)});
    }
    std::vector<int> members;
    for (int i = 0; i < n_jobs; ++i)
      if (same(key_of(plan->jobs[i]), key)) members.push_back(i);
    plan->class_jobs.push_back(members);
    std::stable_sort(work.begin(), work.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    std::vector<int2> items;
    for (const auto& w : work) items.push_back(w.second);
    c.n_items = (int)items.size();
    const int n_state = 1 + 2 * c.groups + c.groups * c.k;
    bool ok = hipMalloc(&c.items, items.size() * sizeof(int2)) == hipSuccess &&
              hipMalloc(&c.state, n_state * sizeof(int)) == hipSuccess &&
              hipMalloc(&c.xbuf, (size_t)c.groups * 4 * key.n * key.n * sizeof(float2)) == hipSuccess &&
              hipMemcpy(c.items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice) == hipSuccess;
    plan->classes.push_back(c);
    if (!ok) { adorym_plan_destroy(plan); return set_err(ctx, ADORYM_EDEVICE, "plan allocation failed"); }
  }
  if (hipMalloc(&plan->d_params, n_jobs * sizeof(MsParams)) != hipSuccess ||
      hipMemcpy(plan->d_params, plan->params.data(), n_jobs * sizeof(MsParams), hipMemcpyHostToDevice) != hipSuccess) {
    adorym_plan_destroy(plan);
    return set_err(ctx, ADORYM_EDEVICE, "plan allocation failed");
  }
  if (plan->classes.size() > 1) {
    bool ok = hipEventCreateWithFlags(&plan->fork, hipEventDisableTiming) == hipSuccess;
    for (const PlanClass& c : plan->classes) {
      if (!ok || c.k != 1) continue;
      hipStream_t s = nullptr;
      hipEvent_t e = nullptr;
      ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
      if (ok) plan->side.push_back(s);
      ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
      if (ok) plan->side_done.push_back(e);
    }
    if (!ok) {
      adorym_plan_destroy(plan);
      return set_err(ctx, ADORYM_EDEVICE, "plan stream creation failed");
    }
  }
  *out = plan;
  return ADORYM_OK;
}

adorym_status adorym_plan_run(adorym_ctx* ctx, adorym_plan* plan) {
  if (!ctx || !plan) return ADORYM_EINVAL;
  hipStream_t st = ctx->stream;
  for (size_t i = 0; i < plan->jobs.size(); ++i) job_prologue(plan->params[i], plan->jobs[i], st);
  const bool timed = ctx->prof && ctx->ev_used + 2 <= (int)ctx->ev.size();
  if (timed) (void)hipEventRecord(ctx->ev[ctx->ev_used], st);
  if (plan->side.empty()) {
    for (const PlanClass& c : plan->classes) class_launch(c, plan->d_params, ctx->d_err, st);
    if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
    for (size_t i = 0; i < plan->jobs.size(); ++i) job_epilogue(plan->params[i], plan->jobs[i], st);
  } else {
    // split classes first, alone (their groups need co-resident workgroups);
    // then every K == 1 class with its jobs' epilogues on its own stream,
    // while the split classes' epilogues run here
    for (const PlanClass& c : plan->classes)
      if (c.k != 1) class_launch(c, plan->d_params, ctx->d_err, st);
    (void)hipEventRecord(plan->fork, st);
    size_t side = 0;
    for (size_t ci = 0; ci < plan->classes.size(); ++ci) {
      const PlanClass& c = plan->classes[ci];
      if (c.k != 1) continue;
      hipStream_t s = plan->side[side];
      (void)hipStreamWaitEvent(s, plan->fork, 0);
      class_launch(c, plan->d_params, ctx->d_err, s);
      for (int i : plan->class_jobs[ci]) job_epilogue(plan->params[i], plan->jobs[i], s);
      (void)hipEventRecord(plan->side_done[side], s);
      ++side;
    }
    for (size_t ci = 0; ci < plan->classes.size(); ++ci)
      if (plan->classes[ci].k != 1)
        for (int i : plan->class_jobs[ci]) job_epilogue(plan->params[i], plan->jobs[i], st);
    for (hipEvent_t e : plan->side_done) (void)hipStreamWaitEvent(st, e, 0);
    if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ADORYM_OK : set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
}

adorym_status adorym_plan_destroy(adorym_plan* plan) {
  if (!plan) return ADORYM_EINVAL;
  for (hipStream_t s : plan->side) (void)hipStreamSynchronize(s);
  for (hipStream_t s : plan->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : plan->side_done) (void)hipEventDestroy(e);
  if (plan->fork) (void)hipEventDestroy(plan->fork);
  for (PlanClass& c : plan->classes) {
    if (c.items) (void)hipFree(c.items);
    if (c.state) (void)hipFree(c.state);
    if (c.xbuf) (void)hipFree(c.xbuf);
  }
  if (plan->d_params) (void)hipFree(plan->d_params);
  delete plan;
  return ADORYM_OK;
}

adorym_status adorym_set_split(adorym_ctx* ctx, int32_t n, int32_t k) {
  if (!ctx) return ADORYM_EINVAL;
  const bool ok = k == 0 || (n == 64 && (k == 1 || k == 2 || k == 4)) ||
                  (n == 96 && (k == 1 || k == 2 || k == 3 || k == 4)) ||
                  (n == 128 && (k == 1 || k == 2 || k == 4 || k == 8)) ||
                  (n == 192 && (k == 2 || k == 4 || k == 6 || k == 8));
  if (!ok) return set_err(ctx, ADORYM_EUNSUPPORTED, "no kernel for this probe size / split");
  if (n == 64) ctx->split64 = k;
  else if (n == 96) ctx->split96 = k;
  else if (n == 128) ctx->split128 = k;
  else ctx->split192 = k;
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
