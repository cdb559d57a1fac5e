// priors.hip -- object priors added to the data loss (Eq. tikhonov, Table
// tab:regularizers): l1, reweighted l1 and total variation, their gradients,
// the adaptive weights of the reweighted l1, and the finite-support
// projection, with their C ABI entry points.
//
// The priors act on two per-voxel quantities: (delta, beta) for refractive-
// index objects, (|O| - mean|O|, arg O) for complex objects (the total
// variation of |O| - mean|O| is that of |O|).  With N_o voxels,
//   R = (1/N_o) sum [a1 W1 |q1| + a2 W2 |q2|]
//     + (gamma/N_o) sum over neighbour pairs along z, y, x of |dq1| + |dq2|
// (W = 1 unless weights are given).  d|t|/dt at t = 0 is taken as 0.
//
// The gradient kernel is one pass over the object, HBM-bound: every
// workgroup owns a 64 x 4 column tile and a run of kZc = 32 slices and
// marches along z (on the 512 x 512 x 128 object, taller tiles lost more to
// the smaller grid than they saved in halo reads); each slice's tile with a
// one-voxel halo is staged in LDS as the two quantities, so x/y neighbours
// come from LDS and z neighbours from the previous step's registers, and
// the next slice's halo is loaded while the current one is processed.  The derivative of a voxel is final once the
// pair with the next slice is known, so each thread writes voxel z-1 while
// it handles slice z; the slices just outside a run are read for the pairs
// that cross its ends (each pair's value is counted by the run holding its
// upper slice).
// Complex objects with an l1 modulus term first reduce mean|O| and the sum of
// the weighted signs (two read-only passes); every reduction is a fixed-order
// FP64 sum (bitwise reproducible).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>

#include <algorithm>

#include "adorym.h"
#include "context.hpp"

namespace {

#ifndef ADORYM_PRIOR_ROWS
#define ADORYM_PRIOR_ROWS 1
#endif
#ifndef ADORYM_PRIOR_ZRUN
#define ADORYM_PRIOR_ZRUN 32
#endif
constexpr int kRows = ADORYM_PRIOR_ROWS;   // rows per thread (256 threads = 64 x 4)
constexpr int kTx = 64, kTy = 4 * kRows, kHx = kTx + 2, kHy = kTy + 2;
constexpr int kHalo = kHx * kHy, kHaloPer = (kHalo + 255) / 256;
constexpr int kZc = ADORYM_PRIOR_ZRUN;     // slices per workgroup
constexpr int kRedBlocks = 1024;           // fixed grid of the reductions

// scalars in the workspace (doubles): [0] mean|O|, [1] mean-term correction
constexpr int kScal = 8;

__device__ __forceinline__ float sgn(float t) { return t > 0.f ? 1.f : (t < 0.f ? -1.f : 0.f); }

__device__ __forceinline__ double block_sum256(double x, double* red) {
  red[threadIdx.x] = x;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Per-voxel quantities (q1, q2) of the priors.
template <int REPR>
__device__ __forceinline__ void quantities(float a, float b, float mean_mod, float& q1, float& q2) {
  if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
    q1 = a;
    q2 = b;
  } else {
    q1 = sqrtf(a * a + b * b) - mean_mod;
    q2 = atan2f(b, a);
  }
}

// (dR/da, dR/db) from (dR/dq1, dR/dq2).
template <int REPR>
__device__ __forceinline__ void chain(float a, float b, float d1, float d2, float& ga, float& gb) {
  if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
    ga = d1;
    gb = d2;
  } else {
    const float m2 = a * a + b * b;
    const float inv2 = m2 > 0.f ? 1.f / m2 : 0.f;
    const float inv = m2 > 0.f ? rsqrtf(m2) : 0.f;
    ga = d1 * a * inv - d2 * b * inv2;
    gb = d1 * b * inv + d2 * a * inv2;
  }
}

struct PriorArgs {
  const float* a; const float* b;
  const float* wa; const float* wb;      // reweighting or null
  float* ga; float* gb;
  int S, Ly, Lx;
  float c1, c2, ctv;                     // a1/N_o, a2/N_o, gamma/N_o
  const double* scal;                    // mean|O|, mean-term correction (complex objects)
  double* part;                          // [gridDim] value partials
  int accumulate;
};

template <int REPR>
__global__ void __launch_bounds__(256) prior_grad_kernel(PriorArgs p) {
  __shared__ float s1[kHy][kHx], s2[kHy][kHx];
  __shared__ double red[256];
  const int tx = threadIdx.x % kTx, ty = threadIdx.x / kTx;    // rows ty + 4 r of the tile
  const int x0 = blockIdx.x * kTx, y0 = blockIdx.y * kTy;
  const int x = x0 + tx;
  const size_t plane = (size_t)p.Ly * p.Lx;
  const float mean_mod = (REPR == ADORYM_OBJ_DELTA_BETA) ? 0.f : (float)p.scal[0];
  const float corr = (REPR == ADORYM_OBJ_DELTA_BETA) ? 0.f : (float)p.scal[1];
  const float ct = p.ctv;
  const int z0 = blockIdx.z * kZc, z1 = min(p.S, z0 + kZc);
  // this thread's halo elements: in-plane offset, -1 outside the object,
  // -2 past the end of the halo
  int hoff[kHaloPer];
#pragma unroll
  for (int u = 0; u < kHaloPer; ++u) {
    const int i = threadIdx.x + 256 * u;
    const int gy = y0 + i / kHx - 1, gx = x0 + i % kHx - 1;
    hoff[u] = i >= kHalo ? -2 : ((gy >= 0 && gy < p.Ly && gx >= 0 && gx < p.Lx) ? gy * p.Lx + gx : -1);
  }
  float na[kHaloPer], nb[kHaloPer];      // the next slice's halo values, loaded a slice ahead
  auto fetch = [&](int z) {
#pragma unroll
    for (int u = 0; u < kHaloPer; ++u) {
      const bool in = hoff[u] >= 0;
      na[u] = in ? p.a[(size_t)z * plane + hoff[u]] : 0.f;
      nb[u] = in ? p.b[(size_t)z * plane + hoff[u]] : 0.f;
    }
  };
  bool mine[kRows];
  float q1p[kRows], q2p[kRows], d1p[kRows], d2p[kRows], ap[kRows], bp[kRows], gpa[kRows], gpb[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int y = y0 + ty + 4 * r;
    mine[r] = x < p.Lx && y < p.Ly;
    q1p[r] = q2p[r] = d1p[r] = d2p[r] = ap[r] = bp[r] = gpa[r] = gpb[r] = 0.f;
    if (mine[r] && z0 > 0) {             // the slice below the run, for the pair (z0-1, z0)
      const size_t i0 = (size_t)(z0 - 1) * plane + (size_t)y * p.Lx + x;
      quantities<REPR>(p.a[i0], p.b[i0], mean_mod, q1p[r], q2p[r]);
    }
  }
  double val = 0.0;
  if (z0 < z1) fetch(z0);
  for (int z = z0; z < z1; ++z) {
    __syncthreads();                     // the last slice's LDS reads are done
#pragma unroll
    for (int u = 0; u < kHaloPer; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (hoff[u] == -2) continue;
      float q1 = 0.f, q2 = 0.f;
      if (hoff[u] >= 0) quantities<REPR>(na[u], nb[u], mean_mod, q1, q2);
      s1[i / kHx][i % kHx] = q1;
      s2[i / kHx][i % kHx] = q2;
    }
    __syncthreads();
    if (z + 1 < z1) fetch(z + 1);        // in flight while this slice is processed
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      if (!mine[r]) continue;
      const int ly = ty + 4 * r, y = y0 + ly;
      const size_t idx = (size_t)z * plane + (size_t)y * p.Lx + x;
      const float q1 = s1[ly + 1][tx + 1], q2 = s2[ly + 1][tx + 1];
      const float w1 = p.wa ? p.wa[idx] : 1.f, w2 = p.wb ? p.wb[idx] : 1.f;
      // l1 (the mean term's own derivative enters through corr)
      float d1 = p.c1 * w1 * sgn(q1) - corr, d2 = p.c2 * w2 * sgn(q2);
      val += (double)(p.c1 * w1 * fabsf(q1) + p.c2 * w2 * fabsf(q2));
      if (ct != 0.f) {
        float tv = 0.f;
        if (x + 1 < p.Lx) {
          const float e1 = s1[ly + 1][tx + 2] - q1, e2 = s2[ly + 1][tx + 2] - q2;
          tv += fabsf(e1) + fabsf(e2);
          d1 -= ct * sgn(e1);
          d2 -= ct * sgn(e2);
        }
        if (x > 0) {
          d1 += ct * sgn(q1 - s1[ly + 1][tx]);
          d2 += ct * sgn(q2 - s2[ly + 1][tx]);
        }
        if (y + 1 < p.Ly) {
          const float e1 = s1[ly + 2][tx + 1] - q1, e2 = s2[ly + 2][tx + 1] - q2;
          tv += fabsf(e1) + fabsf(e2);
          d1 -= ct * sgn(e1);
          d2 -= ct * sgn(e2);
        }
        if (y > 0) {
          d1 += ct * sgn(q1 - s1[ly][tx + 1]);
          d2 += ct * sgn(q2 - s2[ly][tx + 1]);
        }
        if (z > 0) {
          const float e1 = q1 - q1p[r], e2 = q2 - q2p[r];
          tv += fabsf(e1) + fabsf(e2);
          d1 += ct * sgn(e1);
          d2 += ct * sgn(e2);
          d1p[r] -= ct * sgn(e1);
          d2p[r] -= ct * sgn(e2);
        }
        val += (double)(ct * tv);
      }
      if (z > z0) {                      // voxel z-1 is complete
        const size_t ip = idx - plane;
        float ga, gb;
        chain<REPR>(ap[r], bp[r], d1p[r], d2p[r], ga, gb);
        p.ga[ip] = gpa[r] + ga;
        p.gb[ip] = gpb[r] + gb;
      }
      q1p[r] = q1; q2p[r] = q2; d1p[r] = d1; d2p[r] = d2;
      if constexpr (REPR != ADORYM_OBJ_DELTA_BETA) { ap[r] = p.a[idx]; bp[r] = p.b[idx]; }
      // the data gradient this voxel's derivative is added onto, loaded a slice ahead
      gpa[r] = p.accumulate ? p.ga[idx] : 0.f;
      gpb[r] = p.accumulate ? p.gb[idx] : 0.f;
    }
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    if (!mine[r] || z1 <= z0) continue;
    const size_t ip = (size_t)(z1 - 1) * plane + (size_t)(y0 + ty + 4 * r) * p.Lx + x;
    if (z1 < p.S && ct != 0.f) {         // the pair (z1-1, z1) with the slice above the run
      float q1n, q2n;
      quantities<REPR>(p.a[ip + plane], p.b[ip + plane], mean_mod, q1n, q2n);
      d1p[r] -= ct * sgn(q1n - q1p[r]);
      d2p[r] -= ct * sgn(q2n - q2p[r]);
    }
    float ga, gb;
    chain<REPR>(ap[r], bp[r], d1p[r], d2p[r], ga, gb);
    p.ga[ip] = gpa[r] + ga;
    p.gb[ip] = gpb[r] + gb;
  }
  const double tot = block_sum256(val, red);
  if (threadIdx.x == 0) p.part[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

// Fixed-order sum of n partials into *out (times scale); one workgroup.
__global__ void __launch_bounds__(256) finish_sum_kernel(const double* __restrict__ part, int n, double scale,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  const double t = block_sum256(s, red);
  if (threadIdx.x == 0) *out = scale * t;
}

// Complex objects: partial sums of |O| (mode 0) or of W1 sign(|O| - m)
// (mode 1, m = scal[0]) over a fixed grid-stride split.
__global__ void __launch_bounds__(256) modulus_stats_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                            const float* __restrict__ wa, size_t n, int mode,
                                                            const double* __restrict__ scal,
                                                            double* __restrict__ part) {
  __shared__ double red[256];
  const float m = mode ? (float)scal[0] : 0.f;
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float mod = sqrtf(a[i] * a[i] + b[i] * b[i]);
    s += mode ? (double)((wa ? wa[i] : 1.f) * sgn(mod - m)) : (double)mod;
  }
  const double t = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Partial maxima of |q1| and |q2| (weights of the reweighted l1).
template <int REPR>
__global__ void __launch_bounds__(256) quantity_max_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                           size_t n, const double* __restrict__ scal,
                                                           double* __restrict__ part) {
  __shared__ double red[256];
  const float m = (REPR == ADORYM_OBJ_DELTA_BETA) ? 0.f : (float)scal[0];
  float m1 = 0.f, m2 = 0.f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    float q1, q2;
    quantities<REPR>(a[i], b[i], m, q1, q2);
    m1 = fmaxf(m1, fabsf(q1));
    m2 = fmaxf(m2, fabsf(q2));
  }
  for (int k = 0; k < 2; ++k) {
    red[threadIdx.x] = k ? m2 : m1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
      __syncthreads();
    }
    if (threadIdx.x == 0) part[k * kRedBlocks + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) finish_max_kernel(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  for (int k = 0; k < 2; ++k) {
    double m = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += 256) m = fmax(m, part[k * kRedBlocks + i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
    __syncthreads();
  }
}

template <int REPR>
__global__ void weights_kernel(const float* __restrict__ a, const float* __restrict__ b, size_t n,
                               const double* __restrict__ scal, const double* __restrict__ mx, float eps,
                               float* __restrict__ wa, float* __restrict__ wb) {
  const float m = (REPR == ADORYM_OBJ_DELTA_BETA) ? 0.f : (float)scal[0];
  const float m1 = (float)mx[0], m2 = (float)mx[1];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float q1, q2;
    quantities<REPR>(a[i], b[i], m, q1, q2);
    wa[i] = m1 / (fabsf(q1) + eps);
    wb[i] = m2 / (fabsf(q2) + eps);
  }
}

__global__ void support_kernel(const uint8_t* __restrict__ mask, float* __restrict__ a, float* __restrict__ b,
                               size_t n, float vac_a) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    if (!mask[i]) {
      a[i] = vac_a;
      b[i] = 0.f;
    }
  }
}

inline adorym_status fail(adorym_ctx* ctx, adorym_status st, const char* what) {
  if (ctx) snprintf(ctx->msg, sizeof(ctx->msg), "%s", what);
  return st;
}

inline adorym_status launched(adorym_ctx* ctx) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? ADORYM_OK : fail(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
}

inline bool bad_shape(int s, int ly, int lx) { return s < 1 || ly < 1 || lx < 1; }

// workspace: [kScal] scalars, then partials
inline double* scal_of(void* ws) { return static_cast<double*>(ws); }
inline double* part_of(void* ws) { return static_cast<double*>(ws) + kScal; }
inline size_t prior_parts(int s, int ly, int lx) {
  const size_t tiles = (size_t)((lx + kTx - 1) / kTx) * ((ly + kTy - 1) / kTy) * ((s + kZc - 1) / kZc);
  return tiles > 2 * (size_t)kRedBlocks ? tiles : 2 * (size_t)kRedBlocks;
}

// mean|O| into scal[0] (complex objects)
adorym_status mean_modulus(adorym_ctx* ctx, const float* a, const float* b, size_t n, void* ws) {
  hipLaunchKernelGGL(modulus_stats_kernel, dim3(kRedBlocks), dim3(256), 0, ctx->stream, a, b, nullptr, n, 0,
                     scal_of(ws), part_of(ws));
  hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, ctx->stream, part_of(ws), kRedBlocks,
                     1.0 / (double)n, scal_of(ws));
  return launched(ctx);
}

}  // namespace

extern "C" {

size_t adorym_prior_workspace_size(int32_t s, int32_t ly, int32_t lx) {
  if (bad_shape(s, ly, lx)) return 0;
  return (kScal + prior_parts(s, ly, lx)) * sizeof(double);
}

adorym_status adorym_prior_grad(adorym_ctx* ctx, int32_t obj_repr, const float* obj_a, const float* obj_b,
                                int32_t s, int32_t ly, int32_t lx, double l1_a, double l1_b, double tv,
                                const float* w_a, const float* w_b, void* workspace, size_t ws_bytes,
                                double* value, float* g_a, float* g_b, int32_t accumulate) {
  if (!ctx) return ADORYM_EINVAL;
  if (bad_shape(s, ly, lx)) return fail(ctx, ADORYM_EINVAL, "object shape must be positive");
  if (obj_repr != ADORYM_OBJ_DELTA_BETA && obj_repr != ADORYM_OBJ_REAL_IMAG)
    return fail(ctx, ADORYM_EINVAL, "unknown object representation");
  if (!obj_a || !obj_b || !workspace || !value || !g_a || !g_b) return fail(ctx, ADORYM_EINVAL, "NULL array argument");
  if ((w_a == nullptr) != (w_b == nullptr)) return fail(ctx, ADORYM_EINVAL, "w_a and w_b must both be given");
  if (!(l1_a >= 0) || !(l1_b >= 0) || !(tv >= 0)) return fail(ctx, ADORYM_EINVAL, "coefficients must be >= 0");
  if (ws_bytes < adorym_prior_workspace_size(s, ly, lx)) return fail(ctx, ADORYM_ENOMEM, "workspace too small");
  const size_t n = (size_t)s * ly * lx;
  const double inv_n = 1.0 / (double)n;
  hipStream_t st = ctx->stream;
  PriorArgs p{};
  p.a = obj_a; p.b = obj_b; p.wa = w_a; p.wb = w_b; p.ga = g_a; p.gb = g_b;
  p.S = s; p.Ly = ly; p.Lx = lx;
  p.c1 = (float)(l1_a * inv_n); p.c2 = (float)(l1_b * inv_n); p.ctv = (float)(tv * inv_n);
  p.scal = scal_of(workspace);
  p.part = part_of(workspace);
  p.accumulate = accumulate ? 1 : 0;
  if (obj_repr == ADORYM_OBJ_REAL_IMAG) {
    adorym_status r = mean_modulus(ctx, obj_a, obj_b, n, workspace);
    if (r != ADORYM_OK) return r;
    // the mean's own derivative: d/d|O_k| of sum_i c1 W_i |(|O_i| - m)| gets
    // -(1/N_o) sum_i c1 W_i sign(|O_i| - m)
    hipLaunchKernelGGL(modulus_stats_kernel, dim3(kRedBlocks), dim3(256), 0, st, obj_a, obj_b, w_a, n, 1,
                       scal_of(workspace), part_of(workspace));
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, st, part_of(workspace), kRedBlocks,
                       l1_a * inv_n * inv_n, scal_of(workspace) + 1);
  }
  const dim3 grid((lx + kTx - 1) / kTx, (ly + kTy - 1) / kTy, (s + kZc - 1) / kZc);
  if (obj_repr == ADORYM_OBJ_DELTA_BETA)
    hipLaunchKernelGGL(prior_grad_kernel<ADORYM_OBJ_DELTA_BETA>, grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(prior_grad_kernel<ADORYM_OBJ_REAL_IMAG>, grid, dim3(256), 0, st, p);
  hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, st, part_of(workspace),
                     (int)(grid.x * grid.y * grid.z), 1.0, value);
  return launched(ctx);
}

adorym_status adorym_prior_weights(adorym_ctx* ctx, int32_t obj_repr, const float* snap_a, const float* snap_b,
                                   int32_t s, int32_t ly, int32_t lx, double eps, void* workspace, size_t ws_bytes,
                                   float* w_a, float* w_b) {
  if (!ctx) return ADORYM_EINVAL;
  if (bad_shape(s, ly, lx)) return fail(ctx, ADORYM_EINVAL, "object shape must be positive");
  if (obj_repr != ADORYM_OBJ_DELTA_BETA && obj_repr != ADORYM_OBJ_REAL_IMAG)
    return fail(ctx, ADORYM_EINVAL, "unknown object representation");
  if (!snap_a || !snap_b || !workspace || !w_a || !w_b) return fail(ctx, ADORYM_EINVAL, "NULL array argument");
  if (!(eps > 0)) return fail(ctx, ADORYM_EINVAL, "eps must be > 0");
  if (ws_bytes < adorym_prior_workspace_size(s, ly, lx)) return fail(ctx, ADORYM_ENOMEM, "workspace too small");
  const size_t n = (size_t)s * ly * lx;
  hipStream_t st = ctx->stream;
  double* mx = scal_of(workspace) + 2;
  if (obj_repr == ADORYM_OBJ_REAL_IMAG) {
    adorym_status r = mean_modulus(ctx, snap_a, snap_b, n, workspace);
    if (r != ADORYM_OK) return r;
    hipLaunchKernelGGL(quantity_max_kernel<ADORYM_OBJ_REAL_IMAG>, dim3(kRedBlocks), dim3(256), 0, st, snap_a, snap_b,
                       n, scal_of(workspace), part_of(workspace));
  } else {
    hipLaunchKernelGGL(quantity_max_kernel<ADORYM_OBJ_DELTA_BETA>, dim3(kRedBlocks), dim3(256), 0, st, snap_a,
                       snap_b, n, scal_of(workspace), part_of(workspace));
  }
  hipLaunchKernelGGL(finish_max_kernel, dim3(1), dim3(256), 0, st, part_of(workspace), mx);
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  if (obj_repr == ADORYM_OBJ_REAL_IMAG)
    hipLaunchKernelGGL(weights_kernel<ADORYM_OBJ_REAL_IMAG>, dim3(blocks), dim3(256), 0, st, snap_a, snap_b, n,
                       scal_of(workspace), mx, (float)eps, w_a, w_b);
  else
    hipLaunchKernelGGL(weights_kernel<ADORYM_OBJ_DELTA_BETA>, dim3(blocks), dim3(256), 0, st, snap_a, snap_b, n,
                       scal_of(workspace), mx, (float)eps, w_a, w_b);
  return launched(ctx);
}

adorym_status adorym_support_project(adorym_ctx* ctx, int32_t obj_repr, const uint8_t* mask, float* obj_a,
                                     float* obj_b, size_t n) {
  if (!ctx) return ADORYM_EINVAL;
  if (obj_repr != ADORYM_OBJ_DELTA_BETA && obj_repr != ADORYM_OBJ_REAL_IMAG)
    return fail(ctx, ADORYM_EINVAL, "unknown object representation");
  if (!mask || !obj_a || !obj_b) return fail(ctx, ADORYM_EINVAL, "NULL array argument");
  if (n == 0) return ADORYM_OK;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(support_kernel, dim3(blocks), dim3(256), 0, ctx->stream, mask, obj_a, obj_b, n,
                     obj_repr == ADORYM_OBJ_DELTA_BETA ? 0.f : 1.f);
  return launched(ctx);
}

}  // extern "C"
