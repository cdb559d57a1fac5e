// rotate_adam.hip -- tilt-series object rotation (with its exact transpose)
// and the fused Adam update, with their C ABI entry points.
//
// Rotation about the vertical (y) axis, Sec. S1.D.2 "Object orientation",
// Eq. rotation_transform: every xz-plane of the slice-major object [Z][Y][X]
// is resampled at (x0, z0) = R(theta) (x_t - c_x, z_t - c_z) + c with
// bilinear weights, zero outside the array; c = ((Lx-1)/2, (Lz-1)/2).  The
// operation is linear, o_t = R o; the adjoint R^T is computed as a gather
// (each source voxel collects the weights it received), so it is exact and
// deterministic.
//
// Adam (Sec. S1.F, the AdamOptimizer): m = b1 m + (1-b1) g,
// v = b2 v + (1-b2) g^2, x -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>

#include "adorym.h"
#include "context.hpp"

namespace {

struct RotGeom {
  int lz, ly, lx;
  double c, s;        // cos(theta), sin(theta)
  double cz, cx;      // plane centre
};

// Source coordinates of output voxel (zt, xt), FP64.
__device__ __forceinline__ void rot_source(const RotGeom& g, int zt, int xt, double& z0, double& x0) {
  const double dx = (double)xt - g.cx, dz = (double)zt - g.cz;
  x0 = g.c * dx - g.s * dz + g.cx;
  z0 = g.s * dx + g.c * dz + g.cz;
}

// out[zt][y][xt] = sum over the four bilinear taps of in[z][y][x].
__global__ void rotate_kernel(const float* __restrict__ in, float* __restrict__ out, RotGeom g) {
  const size_t plane = (size_t)g.ly * g.lx;
  const size_t total = (size_t)g.lz * plane;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int xt = (int)(i % g.lx);
    const int y = (int)((i / g.lx) % g.ly);
    const int zt = (int)(i / plane);
    double z0, x0;
    rot_source(g, zt, xt, z0, x0);
    const double xf = floor(x0), zf = floor(z0);
    const float wx = (float)(x0 - xf), wz = (float)(z0 - zf);
    const int xi = (int)xf, zi = (int)zf;
    float acc = 0.f;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int zz = zi + dz, xx = xi + dx;
        if (zz >= 0 && zz < g.lz && xx >= 0 && xx < g.lx) {
          const float w = (dz ? wz : 1.f - wz) * (dx ? wx : 1.f - wx);
          acc += w * in[(size_t)zz * plane + (size_t)y * g.lx + xx];
        }
      }
    }
    out[i] = acc;
  }
}

// out[z][y][x] = sum over output voxels (zt, xt) whose taps include (z, x) of
// the tap weight times in[zt][y][xt].  The taps are recomputed exactly as in
// rotate_kernel, so this is the transpose of that operator.
__global__ void rotate_transpose_kernel(const float* __restrict__ in, float* __restrict__ out, RotGeom g) {
  const size_t plane = (size_t)g.ly * g.lx;
  const size_t total = (size_t)g.lz * plane;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % g.lx);
    const int y = (int)((i / g.lx) % g.ly);
    const int z = (int)(i / plane);
    // (zt, xt) has (z, x) among its taps iff its source point lies in
    // [x-1, x+1) x [z-1, z+1): a rotated square centred on the inverse
    // rotation of (x, z), of half-width at most sqrt(2) along each axis
    const double dx = x - g.cx, dz = z - g.cz;
    const double xtc = g.c * dx + g.s * dz + g.cx, ztc = -g.s * dx + g.c * dz + g.cz;
    const int xt0 = (int)floor(xtc - 1.5), zt0 = (int)floor(ztc - 1.5);
    float acc = 0.f;
    for (int zt = zt0; zt <= zt0 + 3; ++zt) {
      if (zt < 0 || zt >= g.lz) continue;
      for (int xt = xt0; xt <= xt0 + 3; ++xt) {
        if (xt < 0 || xt >= g.lx) continue;
        double z0, x0;
        rot_source(g, zt, xt, z0, x0);
        const double xf = floor(x0), zf = floor(z0);
        const int ddx = x - (int)xf, ddz = z - (int)zf;
        if (ddx < 0 || ddx > 1 || ddz < 0 || ddz > 1) continue;
        const float wx = (float)(x0 - xf), wz = (float)(z0 - zf);
        const float w = (ddz ? wz : 1.f - wz) * (ddx ? wx : 1.f - wx);
        acc += w * in[(size_t)zt * plane + (size_t)y * g.lx + xt];
      }
    }
    out[i] = acc;
  }
}

// om1 = 1 - b1 and om2 = 1 - b2 come from the host in FP64 (1 - 0.999f in
// float32 would be off by 1.3e-5 relative).
__global__ void adam_kernel(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, size_t n, float lr, float b1, float om1, float b2, float om2,
                            float eps, float inv_c1, float inv_c2) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + om1 * gi;
    const float vi = b2 * v[i] + om2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    x[i] -= lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
  }
}

// The same step with the iteration count read from device memory when the
// kernel runs (a replayed HIP graph then uses the current count).  Every
// workgroup derives the bias corrections once, in FP64, from b1^t and b2^t
// by repeated squaring; a count below 1 leaves everything unchanged and
// sets an error bit.
constexpr int kErrAdamStep = 8;
__global__ void adam_dev_kernel(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, size_t n, float lr, double b1, double b2, float eps,
                                const int32_t* __restrict__ t_dev, int* __restrict__ err) {
  __shared__ float corr[2];
  const int t = *t_dev;
  if (t < 1) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, kErrAdamStep);
    return;
  }
  if (threadIdx.x == 0) {
    double p1 = 1.0, p2 = 1.0, s1 = b1, s2 = b2;
    for (int e = t; e > 0; e >>= 1) {
      if (e & 1) { p1 *= s1; p2 *= s2; }
      s1 *= s1;
      s2 *= s2;
    }
    corr[0] = (float)(1.0 / (1.0 - p1));
    corr[1] = (float)(1.0 / (1.0 - p2));
  }
  __syncthreads();
  const float inv_c1 = corr[0], inv_c2 = corr[1];
  const float fb1 = (float)b1, om1 = (float)(1.0 - b1), fb2 = (float)b2, om2 = (float)(1.0 - b2);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = fb1 * m[i] + om1 * gi;
    const float vi = fb2 * v[i] + om2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    x[i] -= lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
  }
}

inline int grid_for(size_t n) {
  const size_t blocks = (n + 255) / 256;
  return (int)(blocks < 8192 ? (blocks ? blocks : 1) : 8192);
}

adorym_status rot_err(adorym_ctx* ctx, adorym_status st, const char* what) {
  if (ctx) snprintf(ctx->msg, sizeof(ctx->msg), "%s", what);
  return st;
}

}  // namespace

extern "C" {

adorym_status adorym_rotate(adorym_ctx* ctx, const float* in, float* out, int32_t lz, int32_t ly, int32_t lx,
                            double theta, int transpose) {
  if (!ctx) return ADORYM_EINVAL;
  if (!in || !out) return rot_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (in == out) return rot_err(ctx, ADORYM_EINVAL, "rotation cannot run in place");
  if (lz < 1 || ly < 1 || lx < 1) return rot_err(ctx, ADORYM_EINVAL, "sizes must be >= 1");
  RotGeom g{lz, ly, lx, cos(theta), sin(theta), (lz - 1) / 2.0, (lx - 1) / 2.0};
  const size_t n = (size_t)lz * ly * lx;
  if (transpose)
    hipLaunchKernelGGL(rotate_transpose_kernel, dim3(grid_for(n)), dim3(256), 0, ctx->stream, in, out, g);
  else
    hipLaunchKernelGGL(rotate_kernel, dim3(grid_for(n)), dim3(256), 0, ctx->stream, in, out, g);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ADORYM_OK : rot_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
}

adorym_status adorym_adam(adorym_ctx* ctx, float* x, const float* g, float* m, float* v, size_t n, double lr,
                          double beta1, double beta2, double eps, int32_t t) {
  if (!ctx) return ADORYM_EINVAL;
  if (!x || !g || !m || !v) return rot_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (t < 1) return rot_err(ctx, ADORYM_EINVAL, "iteration count t must be >= 1");
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return rot_err(ctx, ADORYM_EINVAL, "need 0 <= beta < 1 and eps > 0");
  if (n == 0) return ADORYM_OK;
  const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, ctx->stream, x, g, m, v, n, (float)lr,
                     (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), (float)eps,
                     (float)(1.0 / c1), (float)(1.0 / c2));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ADORYM_OK : rot_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
}

adorym_status adorym_adam_dev(adorym_ctx* ctx, float* x, const float* g, float* m, float* v, size_t n, double lr,
                              double beta1, double beta2, double eps, const int32_t* t) {
  if (!ctx) return ADORYM_EINVAL;
  if (!x || !g || !m || !v || !t) return rot_err(ctx, ADORYM_EINVAL, "NULL array argument");
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return rot_err(ctx, ADORYM_EINVAL, "need 0 <= beta < 1 and eps > 0");
  if (n == 0) return ADORYM_OK;
  hipLaunchKernelGGL(adam_dev_kernel, dim3(grid_for(n)), dim3(256), 0, ctx->stream, x, g, m, v, n, (float)lr,
                     beta1, beta2, (float)eps, t, ctx->d_err);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ADORYM_OK : rot_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
}

}  // extern "C"
