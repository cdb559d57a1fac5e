// multislice.hip -- fused multislice forward / loss / adjoint kernels and the
// C ABI entry points adorym_forward and adorym_loss_grad.
//
// One workgroup per scan position does everything for that position:
//   probe placement by Fourier shift (Eq. fourier_shift),
//   S slice modulations (Eq. ri_modulation / complex_modulation) with S - 1
//   paraxial Fresnel propagations (Eqs. fresnel_prop, paraxial_kernel),
//   the Fraunhofer far field (Eq. fraunhofer) and |Psi|^2,
//   the loss (Eq. lsq_loss or poisson_loss) and its residual,
//   and the reverse sweep giving dL/d(object), dL/d(probe), dL/d(shift).
// Steps follow Alg. 1 (TakeObjectChunk, FourierShift, MultislicePropagate,
// FarFieldPropagate).  The wave stays in registers for the whole sweep; the
// object is read straight from HBM slice by slice and its gradient is
// scattered with float atomics.  The reverse sweep rebuilds the wave
// entering each slice by stepping the forward recursion backwards
// (psi_{j-1} = t_{j-1}^{-1} P^H psi_j), and re-anchors it on checkpoints of
// the forward sweep stored every ckpt_every slices.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/adorym.h"
#include "fastmath.hpp"
#include "tile.hpp"

using namespace adorym;

#ifndef ADORYM_L128
#define ADORYM_L128 8
#endif

struct adorym_ctx {
  int device;
  hipStream_t stream;
  int* d_err;          // deferred device error flags (bit 0: chunk out of range)
  char msg[512];
  // optional timing of the main multislice kernel (adorym_profile_*)
  std::vector<hipEvent_t> ev;   // start/stop pairs
  int ev_used = 0;
  bool prof = false;
};

namespace {

struct MsParams {
  const float* a;          // delta or Re O, [S][Ly][Lx]
  const float* b;          // beta or Im O
  const float2* q;         // probe spectrum DFT(p)/N^2, thread-native COL/spectral layout
  const int32_t* corner;   // [B][2]
  const float* shift;      // [B][2]
  const float* i_meas;     // [B][N][N]
  float* intensity;        // [B][N][N] or null
  float* g_a;              // [S][Ly][Lx] or null
  float* g_b;
  float* g_shift;          // [B][2] or null
  float2* ckpt;            // [B][nslots][R*THREADS]
  float2* gacc;            // [B][R*THREADS] or null (probe-gradient partials)
  double* loss_part;       // [B]
  int* err;
  int S, Ly, Lx, ckpt_every, nslots;
  int loss, obj_repr, accumulate;
  float kdz;               // k * dz
  double chirp;            // lambda dz / dx^2
  double eps;
  double inv_n;            // 1 / (B N^2)
};

__device__ __forceinline__ bool is_ckpt(int j, int S, int C) { return (j % C == 0) || (j == S - 1); }
__device__ __forceinline__ int ckpt_slot(int j, int S, int C) {
  return (j % C == 0) ? j / C : (S - 1) / C + 1;
}

// fftfreq(N) in cycles/pixel for natural index k
template <int N>
__device__ __forceinline__ double freq(int k) {
  return double(k < (N + 1) / 2 ? k : k - N) / double(N);
}

// Transmission t and its inverse for one voxel (REPR = ADORYM_OBJ_*).
template <int REPR>
__device__ __forceinline__ void transmission(float kdz, float a, float b, float2& t, float2& tinv) {
  if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
    float s, c;
    sincos_f32(kdz * a, s, c);
    const float v = kdz * b;
    const float att = exp_f32(-v), gain = exp_f32(v);
    t = make_float2(c * att, s * att);
    tinv = make_float2(c * gain, -s * gain);
  } else {
    t = make_float2(a, b);
    const float inv = 1.0f / (a * a + b * b);
    tinv = make_float2(a * inv, -b * inv);
  }
}

// Element coordinates (y, x) of register m in ROW (line = y) or COL layout.
template <class C, bool ROW>
__device__ __forceinline__ void coord_nat(const Lane<C>& ln, int m, int& y, int& x) {
  if (ROW) { y = ln.line; x = ln.pos_nat(m); }
  else     { y = ln.pos_nat(m); x = ln.line; }
}

// Shared memory of the multislice kernel.
template <class C>
struct MsShared {
  float2 buf[C::LDS_FIELD];
  Tables<C> tb;
  float2 ey[C::N];     // exp(-2 pi i s_y f(k)), natural k
  float2 ex[C::N];
  double red[2 * C::WAVES];
};

template <class C>
__device__ __forceinline__ void setup_tables(MsShared<C>& sh, const Lane<C>& ln, double chirp, float sy, float sx) {
  build_twiddles<C>(sh.tb, ln.tid);
  build_fresnel<C>(sh.tb, ln.tid, chirp);
  for (int k = ln.tid; k < C::N; k += C::THREADS) {
    double f = freq<C::N>(k), s, c;
    sincospi(-2.0 * double(sy) * f, &s, &c);
    sh.ey[k] = make_float2(float(c), float(s));
    sincospi(-2.0 * double(sx) * f, &s, &c);
    sh.ex[k] = make_float2(float(c), float(s));
  }
  __syncthreads();
}

// Per-thread byte offsets of the chunk elements inside one object slice.
//   ROW layout: element m at row_off + 4 L m         (immediate offsets)
//   COL layout: element m at col_off + m * col_step  (uniform step in an SGPR)
struct ChunkOffsets {
  uint32_t row_off, col_off, col_step, slice_bytes;
};

template <class C>
__device__ __forceinline__ ChunkOffsets chunk_offsets(const Lane<C>& ln, int cy, int cx, int Ly, int Lx) {
  ChunkOffsets o;
  o.row_off = (uint32_t)(((cy + ln.line) * Lx + cx + ln.q) * 4);
  o.col_off = (uint32_t)(((cy + ln.q) * Lx + cx + ln.line) * 4);
  o.col_step = (uint32_t)(4 * C::L * Lx);
  o.slice_bytes = (uint32_t)((size_t)Ly * Lx * 4);
  return o;
}

template <class C, bool ROW>
__device__ __forceinline__ float chunk_load(rsrc_t r, const ChunkOffsets& o, int m) {
  return ROW ? bload(r, o.row_off + 4 * C::L * m, 0) : bload(r, o.col_off, (uint32_t)m * o.col_step);
}
template <class C, bool ROW>
__device__ __forceinline__ void chunk_atomic_add(rsrc_t r, const ChunkOffsets& o, int m, float v) {
  if (ROW) batomic_add(r, v, o.row_off + 4 * C::L * m, 0);
  else batomic_add(r, v, o.col_off, (uint32_t)m * o.col_step);
}

__device__ __forceinline__ rsrc_t slice_rsrc(const float* base, int j, const ChunkOffsets& o) {
  return make_rsrc(base + (size_t)j * (o.slice_bytes / 4), o.slice_bytes);
}

// Modulate the wave by slice j (Eq. ri_modulation or complex_modulation).
template <class C, int REPR, bool ROW>
__device__ __forceinline__ void modulate(float2 (&v)[C::R], const MsParams& P, const ChunkOffsets& o, int j) {
  const rsrc_t ra = slice_rsrc(P.a, j, o), rb = slice_rsrc(P.b, j, o);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    float2 t, tinv;
    transmission<REPR>(P.kdz, chunk_load<C, ROW>(ra, o, m), chunk_load<C, ROW>(rb, o, m), t, tinv);
    v[m] = cmul(v[m], t);
  }
}

// Thread-native storage of a whole field: element m of thread tid at
// (m * THREADS + tid) float2 slots.
template <class C>
__device__ __forceinline__ void field_store(const float2 (&v)[C::R], float2* base, const Lane<C>& ln) {
  const rsrc_t r = make_rsrc(base, C::R * C::THREADS * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) bstore2(r, v[m], ln.tid * 8, m * C::THREADS * 8);
}
template <class C>
__device__ __forceinline__ void field_load(float2 (&v)[C::R], const float2* base, const Lane<C>& ln) {
  const rsrc_t r = make_rsrc(base, C::R * C::THREADS * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) v[m] = bload2(r, ln.tid * 8, m * C::THREADS * 8);
}

template <class C>
__device__ __forceinline__ float2* ckpt_ptr(const MsParams& P, int b, int slot) {
  return P.ckpt + ((size_t)b * P.nslots + slot) * (C::R * C::THREADS);
}

// psi_0 = IDFT(Q * e_b): Q is in COL layout (line kx natural, pos ky spectral).
template <class C>
__device__ __forceinline__ void place_probe(float2 (&v)[C::R], const MsParams& P, MsShared<C>& sh, const Lane<C>& ln) {
  const float2 exv = sh.ex[ln.line];
  field_load<C>(v, P.q, ln);
#pragma unroll
  for (int m = 0; m < C::R; ++m) v[m] = cmul(v[m], cmul(sh.ey[ln.pos_spec(m)], exv));
  ifft_line<C, +1>(v, sh.tb, ln);                 // along y -> natural
  transpose<C>(v, sh.buf, ln, false, true);       // -> ROW, x spectral
  ifft_line<C, +1>(v, sh.tb, ln);                 // along x -> natural
}

// One forward slice step: (store) modulate, and propagate to slice j + 1.
template <class C, int REPR, bool ROW, bool CKPT>
__device__ __forceinline__ void forward_slice(float2 (&v)[C::R], const MsParams& P, MsShared<C>& sh,
                                              const Lane<C>& ln, const ChunkOffsets& o, int b, int j) {
  if (CKPT && is_ckpt(j, P.S, P.ckpt_every)) field_store<C>(v, ckpt_ptr<C>(P, b, ckpt_slot(j, P.S, P.ckpt_every)), ln);
  modulate<C, REPR, ROW>(v, P, o, j);
  if (j < P.S - 1) {
    propagate_line<C, false>(v, sh.tb, ln);
    transpose<C>(v, sh.buf, ln, false, false);
    propagate_line<C, false>(v, sh.tb, ln);
  }
}

// Reverse slice step j (layout ROW/COL): gradient of slice j, then the two
// fields are taken back to slice j-1 by the adjoint propagator.
//   in : psi = phi_j (the wave leaving slice j, rebuilt by the backward
//        recursion) unless slice j is anchored on a checkpoint;
//        lam = dL/dphi_j
//   out: psi = phi_{j-1} = P^H psi_j, lam = dL/dphi_{j-1} = P^H conj(t_j) lam
template <class C, int REPR, bool ROW>
__device__ __forceinline__ void backward_slice(float2 (&psi)[C::R], float2 (&lam)[C::R], const MsParams& P,
                                               MsShared<C>& sh, const Lane<C>& ln, const ChunkOffsets& o, int b,
                                               int j) {
  const bool anchored = is_ckpt(j, P.S, P.ckpt_every);
  if (anchored) field_load<C>(psi, ckpt_ptr<C>(P, b, ckpt_slot(j, P.S, P.ckpt_every)), ln);  // psi_j exactly
  const rsrc_t ra = slice_rsrc(P.a, j, o), rb = slice_rsrc(P.b, j, o);
  const bool grads = P.g_a != nullptr;
  const rsrc_t rga = grads ? slice_rsrc(P.g_a, j, o) : ra;
  const rsrc_t rgb = grads ? slice_rsrc(P.g_b, j, o) : rb;
  const float kdz = P.kdz;
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    float2 t, tinv;
    transmission<REPR>(kdz, chunk_load<C, ROW>(ra, o, m), chunk_load<C, ROW>(rb, o, m), t, tinv);
    const float2 in_wave = anchored ? psi[m] : cmul(psi[m], tinv);   // psi_j
    const float2 out_wave = anchored ? cmul(psi[m], t) : psi[m];     // phi_j
    const float2 l = lam[m];
    if (grads) {
      if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
        const float2 z = cmulc(l, out_wave);          // conj(phi) lam (imag part sign: lam conj(phi))
        chunk_atomic_add<C, ROW>(rga, o, m, kdz * z.y);
        chunk_atomic_add<C, ROW>(rgb, o, m, -kdz * z.x);
      } else {
        const float2 z = cmulc(l, in_wave);           // conj(psi) lam
        chunk_atomic_add<C, ROW>(rga, o, m, z.x);
        chunk_atomic_add<C, ROW>(rgb, o, m, z.y);
      }
    }
    lam[m] = cmulc(l, t);                              // conj(t) lam = dL/dpsi_j
    psi[m] = in_wave;
  }
  if (j > 0) {
    const bool need_psi = !is_ckpt(j - 1, P.S, P.ckpt_every);
    if (need_psi) propagate_line<C, true>(psi, sh.tb, ln);
    propagate_line<C, true>(lam, sh.tb, ln);
    if (need_psi) transpose<C>(psi, sh.buf, ln, false, false);
    transpose<C>(lam, sh.buf, ln, false, false);
    if (need_psi) propagate_line<C, true>(psi, sh.tb, ln);
    propagate_line<C, true>(lam, sh.tb, ln);
  }
}

#ifdef ADORYM_DEBUG_STAGE
#define DEBUG_DUMP(k, v) \
  if (ADORYM_DEBUG_STAGE == (k)) field_store<C>((v), P.ckpt + (size_t)b * (C::R * C::THREADS), ln)
#else
#define DEBUG_DUMP(k, v)
#endif

template <class C, int REPR, int LOSSK, bool LOSS>
__global__ void __launch_bounds__(C::THREADS) multislice_kernel(MsParams P) {
  __shared__ MsShared<C> sh;
  const Lane<C> ln(threadIdx.x);
  const int b = blockIdx.x;
  const int cy = P.corner[2 * b], cx = P.corner[2 * b + 1];
  const float sy = P.shift[2 * b], sx = P.shift[2 * b + 1];
  constexpr int N = C::N;
  constexpr int NN = N * N;

  // TakeObjectChunk: the chunk must lie inside the object.
  if (cy < 0 || cx < 0 || cy + N > P.Ly || cx + N > P.Lx) {
    if (threadIdx.x == 0) atomicOr(P.err, 1);
    if (LOSS) {
      if (threadIdx.x == 0) P.loss_part[b] = 0.0;
      if (P.gacc)
        for (int i = threadIdx.x; i < NN; i += C::THREADS) P.gacc[(size_t)b * NN + i] = make_float2(0.f, 0.f);
      if (P.g_shift && !P.accumulate && threadIdx.x < 2) P.g_shift[2 * b + threadIdx.x] = 0.f;
    }
    if (P.intensity)
      for (int i = threadIdx.x; i < NN; i += C::THREADS) P.intensity[(size_t)b * NN + i] = 0.f;
    return;
  }

  setup_tables<C>(sh, ln, P.chirp, sy, sx);
  const ChunkOffsets o = chunk_offsets<C>(ln, cy, cx, P.Ly, P.Lx);

  float2 v[C::R];
  place_probe<C>(v, P, sh, ln);
  DEBUG_DUMP(1, v);

  // MultislicePropagate: even slices in ROW layout, odd slices in COL layout.
  for (int j = 0; j < P.S; j += 2) {
    forward_slice<C, REPR, true, LOSS>(v, P, sh, ln, o, b, j);
    if (j + 1 < P.S) forward_slice<C, REPR, false, LOSS>(v, P, sh, ln, o, b, j + 1);
  }
  const bool last_row = ((P.S - 1) & 1) == 0;
  DEBUG_DUMP(2, v);

  // FarFieldPropagate: inverse DFT along the current lines, transpose, along
  // the other axis.  Result: spectral along the lines of the final layout.
  fft_line<C, +1>(v, sh.tb, ln);
  DEBUG_DUMP(3, v);
  transpose<C>(v, sh.buf, ln, true, false);
  DEBUG_DUMP(4, v);
  fft_line<C, +1>(v, sh.tb, ln);
  DEBUG_DUMP(5, v);
  const float inv_nf = 1.0f / float(N);

  // Stage the measured pattern (or prepare the intensity output) in LDS.
  float* fb = reinterpret_cast<float*>(sh.buf);
  constexpr int PF = N + 1;
  __syncthreads();
  if (LOSS) {
    const float* im = P.i_meas + (size_t)b * NN;
    for (int i = threadIdx.x; i < NN; i += C::THREADS) fb[(i / N) * PF + (i % N)] = im[i];
    __syncthreads();
  }
  // Per-pixel loss terms in FP32; the sum over pixels is accumulated in FP64.
  double lsum = 0.0;
  float ireg[C::R];
  const float eps = (float)P.eps;
  const float inv_n = (float)P.inv_n;
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    int ky, kx;
    if (last_row) { ky = ln.pos_spec(m); kx = ln.line; }    // final layout COL
    else          { ky = ln.line; kx = ln.pos_spec(m); }    // final layout ROW
    const float2 psi_det = cscale(v[m], inv_nf);
    const float ip = psi_det.x * psi_det.x + psi_det.y * psi_det.y;
    ireg[m] = ip;
    if (LOSS) {
      const int dy = (ky + N / 2) % N, dx = (kx + N / 2) % N;
      const float imv = fb[dy * PF + dx];
      float term, dldi;
      if constexpr (LOSSK == ADORYM_LOSS_GAUSSIAN) {
        const float sp = sqrtf(ip + eps), sm = sqrtf(imv + eps);
        term = (sp - sm) * (sp - sm);
        dldi = (1.0f - sm / sp) * inv_n;
      } else {
        term = ip - imv * logf(ip + eps);
        dldi = (1.0f - imv / (ip + eps)) * inv_n;
      }
      lsum += (double)term;
      // far-field residual 2 dL/dI Psi, scaled by 1/N for the adjoint DFT
      v[m] = cscale(psi_det, 2.0f * dldi * inv_nf);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (P.intensity) {
    __syncthreads();   // every thread is done reading the measured pattern
#pragma unroll
    for (int m = 0; m < C::R; ++m) {
      int ky, kx;
      if (last_row) { ky = ln.pos_spec(m); kx = ln.line; }
      else          { ky = ln.line; kx = ln.pos_spec(m); }
      fb[((ky + N / 2) % N) * PF + ((kx + N / 2) % N)] = ireg[m];
    }
    __syncthreads();
    float* out = P.intensity + (size_t)b * NN;
    for (int i = threadIdx.x; i < NN; i += C::THREADS) out[i] = fb[(i / N) * PF + (i % N)];
  }
  if (!LOSS) return;

  {
    double tot = block_sum<C::THREADS>(lsum, sh.red);
    if (threadIdx.x == 0) P.loss_part[b] = tot * P.inv_n;   // mean over the B N^2 pixels
  }

  // Adjoint of the far field: DFT back along the two axes.
  ifft_line<C, -1>(v, sh.tb, ln);
  transpose<C>(v, sh.buf, ln, false, true);
  ifft_line<C, -1>(v, sh.tb, ln);
  // v = lambda_{S-1} in the layout of slice S-1

  float2 psi[C::R];
  int j = P.S - 1;
  if (!last_row) {
    backward_slice<C, REPR, false>(psi, v, P, sh, ln, o, b, j);
    --j;
  }
  // now slice j is even (ROW); pairs (j ROW, j-1 COL) down to slice 0
  for (; j >= 1; j -= 2) {
    backward_slice<C, REPR, true>(psi, v, P, sh, ln, o, b, j);
    backward_slice<C, REPR, false>(psi, v, P, sh, ln, o, b, j - 1);
  }
  if (j == 0) backward_slice<C, REPR, true>(psi, v, P, sh, ln, o, b, 0);
  // v = dL/d(shifted probe) in ROW layout, natural order.

  // FourierShift adjoint: G = DFT(g_pb) in COL layout (kx line, ky spectral).
  fft_line<C, -1>(v, sh.tb, ln);
  transpose<C>(v, sh.buf, ln, true, false);
  fft_line<C, -1>(v, sh.tb, ln);
  const float2 exv = sh.ex[ln.line];
  const double fx = freq<N>(ln.line);
  double gsy = 0.0, gsx = 0.0;
  const rsrc_t rq = make_rsrc(P.q, C::R * C::THREADS * 8);
  const rsrc_t rg = make_rsrc(P.gacc ? P.gacc + (size_t)b * NN : P.q, C::R * C::THREADS * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const int ky = ln.pos_spec(m);
    const float2 e = cmul(sh.ey[ky], exv);
    const float2 g = v[m];
    if (P.gacc) bstore2(rg, cmulc(g, e), ln.tid * 8, m * C::THREADS * 8);
    const float2 qv = bload2(rq, ln.tid * 8, m * C::THREADS * 8);
    const float2 z = cmul(cmulc(qv, g), e);     // conj(G) Q e
    gsy += freq<N>(ky) * double(z.y);
    gsx += fx * double(z.y);
  }
  if (P.g_shift) {
    double ty = block_sum<C::THREADS>(gsy, sh.red);
    double tx = block_sum<C::THREADS>(gsx, sh.red + C::WAVES);
    if (threadIdx.x == 0) {
      const double two_pi = 6.283185307179586476925286766559;
      float vy = float(two_pi * ty), vx = float(two_pi * tx);
      if (P.accumulate) { P.g_shift[2 * b] += vy; P.g_shift[2 * b + 1] += vx; }
      else { P.g_shift[2 * b] = vy; P.g_shift[2 * b + 1] = vx; }
    }
  }
}

// Probe spectrum Q = DFT(p) / N^2 in the thread-native COL/spectral layout.
template <class C>
__global__ void __launch_bounds__(C::THREADS) probe_spectrum_kernel(const float2* __restrict__ probe,
                                                                    float2* __restrict__ q) {
  __shared__ float2 buf[C::LDS_FIELD];
  __shared__ Tables<C> tb;
  const Lane<C> ln(threadIdx.x);
  build_twiddles<C>(tb, ln.tid);
  __syncthreads();
  constexpr int N = C::N;
  float2 v[C::R];
#pragma unroll
  for (int m = 0; m < C::R; ++m) v[m] = probe[ln.line * N + ln.pos_nat(m)];
  fft_line<C, -1>(v, tb, ln);
  transpose<C>(v, buf, ln, true, false);
  fft_line<C, -1>(v, tb, ln);
  const float s = 1.0f / float(N * N);
#pragma unroll
  for (int m = 0; m < C::R; ++m) q[m * C::THREADS + ln.tid] = cscale(v[m], s);
}

// Loss total and probe gradient g_p = IDFT(sum_b G_b conj(e_b)) / N^2.
template <class C>
__global__ void __launch_bounds__(C::THREADS) finalize_kernel(const double* __restrict__ loss_part, int nb,
                                                              double* __restrict__ loss,
                                                              const float2* __restrict__ gacc,
                                                              float2* __restrict__ g_probe, int accumulate) {
  __shared__ float2 buf[C::LDS_FIELD];
  __shared__ Tables<C> tb;
  const Lane<C> ln(threadIdx.x);
  constexpr int N = C::N, NN = N * N;
  if (threadIdx.x == 0 && loss) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += loss_part[i];   // fixed order
    *loss = s;
  }
  if (!g_probe) return;
  build_twiddles<C>(tb, ln.tid);
  __syncthreads();
  float2 v[C::R];
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    float sx = 0.f, sy = 0.f;
    for (int i = 0; i < nb; ++i) {
      float2 t = gacc[(size_t)i * NN + m * C::THREADS + ln.tid];
      sx += t.x; sy += t.y;
    }
    v[m] = make_float2(sx, sy);
  }
  ifft_line<C, +1>(v, tb, ln);
  transpose<C>(v, buf, ln, false, true);
  ifft_line<C, +1>(v, tb, ln);
  const float s = 1.0f / float(NN);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const int idx = ln.line * N + ln.pos_nat(m);
    float2 g = cscale(v[m], s);
    if (accumulate) g = cadd(g, g_probe[idx]);
    g_probe[idx] = g;
  }
}

__global__ void fill_kernel(float* __restrict__ p, size_t n, float val) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = val;
}

// ----------------------------------------------------------------------------
// Host side
// ----------------------------------------------------------------------------
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct WsLayout {
  size_t q, loss_part, gacc, ckpt, total;
  int nslots;
};

WsLayout ws_layout(const adorym_geom* g, int batch) {
  WsLayout w{};
  const size_t nn = (size_t)g->n * g->n;
  const int S = g->n_slices, C = g->ckpt_every;
  w.nslots = (S - 1) / C + 1 + (((S - 1) % C) != 0 ? 1 : 0);
  size_t off = 0;
  w.q = off; off += align256(nn * sizeof(float2));
  w.loss_part = off; off += align256((size_t)batch * sizeof(double));
  w.gacc = off; off += align256((size_t)batch * nn * sizeof(float2));
  w.ckpt = off; off += align256((size_t)batch * w.nslots * nn * sizeof(float2));
  w.total = off;
  return w;
}

adorym_status set_err(adorym_ctx* ctx, adorym_status st, const char* what) {
  if (ctx) snprintf(ctx->msg, sizeof(ctx->msg), "%s", what);
  return st;
}

adorym_status check_geom(adorym_ctx* ctx, const adorym_geom* g, int batch) {
  if (!ctx) return ADORYM_EINVAL;
  if (!g) return set_err(ctx, ADORYM_EINVAL, "geometry is NULL");
  if (!adorym_supports_n(g->n)) return set_err(ctx, ADORYM_EUNSUPPORTED, "probe size N has no kernel");
  if (g->n_slices < 1) return set_err(ctx, ADORYM_EINVAL, "n_slices must be >= 1");
  if (g->obj_ny < g->n || g->obj_nx < g->n) return set_err(ctx, ADORYM_EINVAL, "object smaller than the probe");
  if (g->ckpt_every < 1) return set_err(ctx, ADORYM_EINVAL, "ckpt_every must be >= 1");
  if (!(g->wavelength_m > 0) || !(g->pixel_m > 0) || !(g->slice_dz_m >= 0))
    return set_err(ctx, ADORYM_EINVAL, "wavelength, pixel and slice spacing must be positive");
  if (g->loss != ADORYM_LOSS_GAUSSIAN && g->loss != ADORYM_LOSS_POISSON)
    return set_err(ctx, ADORYM_EINVAL, "unknown loss");
  if (g->obj_repr != ADORYM_OBJ_DELTA_BETA && g->obj_repr != ADORYM_OBJ_REAL_IMAG)
    return set_err(ctx, ADORYM_EINVAL, "unknown object representation");
  if (!(g->eps >= 0)) return set_err(ctx, ADORYM_EINVAL, "eps must be >= 0");
  if (batch < 1) return set_err(ctx, ADORYM_EINVAL, "batch must be >= 1");
  return ADORYM_OK;
}

void fill(hipStream_t st, float* p, size_t n, float v) {
  if (!p || n == 0) return;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, st, p, n, v);
}

template <class C, bool LOSS>
void launch_ms(const MsParams& P, int repr, int lossk, int batch, hipStream_t st) {
  const dim3 grid(batch), block(C::THREADS);
  if (repr == ADORYM_OBJ_DELTA_BETA) {
    if (lossk == ADORYM_LOSS_GAUSSIAN)
      hipLaunchKernelGGL((multislice_kernel<C, ADORYM_OBJ_DELTA_BETA, ADORYM_LOSS_GAUSSIAN, LOSS>), grid, block, 0, st, P);
    else
      hipLaunchKernelGGL((multislice_kernel<C, ADORYM_OBJ_DELTA_BETA, ADORYM_LOSS_POISSON, LOSS>), grid, block, 0, st, P);
  } else {
    if (lossk == ADORYM_LOSS_GAUSSIAN)
      hipLaunchKernelGGL((multislice_kernel<C, ADORYM_OBJ_REAL_IMAG, ADORYM_LOSS_GAUSSIAN, LOSS>), grid, block, 0, st, P);
    else
      hipLaunchKernelGGL((multislice_kernel<C, ADORYM_OBJ_REAL_IMAG, ADORYM_LOSS_POISSON, LOSS>), grid, block, 0, st, P);
  }
}

template <class C>
adorym_status run(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                  const int32_t* corner, const float* shift, int batch, const float* i_meas, void* ws,
                  double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift, float* intensity,
                  bool with_loss) {
  const WsLayout w = ws_layout(g, batch);
  char* base = static_cast<char*>(ws);
  MsParams P{};
  P.a = a; P.b = b;
  P.q = reinterpret_cast<const float2*>(base + w.q);
  P.corner = corner; P.shift = shift; P.i_meas = i_meas; P.intensity = intensity;
  P.g_a = g_a; P.g_b = g_b; P.g_shift = g_shift;
  P.ckpt = reinterpret_cast<float2*>(base + w.ckpt);
  P.gacc = g_probe ? reinterpret_cast<float2*>(base + w.gacc) : nullptr;
  P.loss_part = reinterpret_cast<double*>(base + w.loss_part);
  P.err = ctx->d_err;
  P.S = g->n_slices; P.Ly = g->obj_ny; P.Lx = g->obj_nx;
  P.ckpt_every = g->ckpt_every; P.nslots = w.nslots;
  P.loss = g->loss; P.obj_repr = g->obj_repr;
  P.accumulate = (g->flags & ADORYM_ACCUMULATE_GRADS) ? 1 : 0;
  P.kdz = (float)(2.0 * M_PI / g->wavelength_m * g->slice_dz_m);
  P.chirp = g->wavelength_m * g->slice_dz_m / (g->pixel_m * g->pixel_m);
  P.eps = g->eps;
  P.inv_n = 1.0 / ((double)batch * g->n * g->n);

  hipStream_t st = ctx->stream;
  const bool timed = ctx->prof && ctx->ev_used + 2 <= (int)ctx->ev.size();
  hipLaunchKernelGGL((probe_spectrum_kernel<C>), dim3(1), dim3(C::THREADS), 0, st,
                     reinterpret_cast<const float2*>(probe), const_cast<float2*>(P.q));
  if (with_loss) {
    const size_t nobj = (size_t)g->n_slices * g->obj_ny * g->obj_nx;
    if (!P.accumulate) {
      if (g_a) fill(st, g_a, nobj, 0.f);
      if (g_b) fill(st, g_b, nobj, 0.f);
    }
    if (timed) (void)hipEventRecord(ctx->ev[ctx->ev_used], st);
    launch_ms<C, true>(P, g->obj_repr, g->loss, batch, st);
    if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
    hipLaunchKernelGGL((finalize_kernel<C>), dim3(1), dim3(C::THREADS), 0, st, P.loss_part, batch, loss,
                       P.gacc, reinterpret_cast<float2*>(g_probe), P.accumulate);
  } else {
    if (timed) (void)hipEventRecord(ctx->ev[ctx->ev_used], st);
    launch_ms<C, false>(P, g->obj_repr, g->loss, batch, st);
    if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return ADORYM_OK;
}

using Cfg64 = TileCfg<64, 4>;
using Cfg128 = TileCfg<128, ADORYM_L128>;

adorym_status dispatch(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                       const int32_t* corner, const float* shift, int batch, const float* i_meas, void* ws,
                       double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift, float* intensity,
                       bool with_loss) {
  switch (g->n) {
    case 64: return run<Cfg64>(ctx, g, a, b, probe, corner, shift, batch, i_meas, ws, loss, g_a, g_b, g_probe,
                               g_shift, intensity, with_loss);
    case 128: return run<Cfg128>(ctx, g, a, b, probe, corner, shift, batch, i_meas, ws, loss, g_a, g_b, g_probe,
                                 g_shift, intensity, with_loss);
    default: return set_err(ctx, ADORYM_EUNSUPPORTED, "probe size N has no kernel");
  }
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
  if (flag & 1) return set_err(ctx, ADORYM_ERANGE, "a chunk left the object; those positions contributed nothing");
  return ADORYM_OK;
}

const char* adorym_last_error_message(adorym_ctx* ctx) { return ctx ? ctx->msg : "no context"; }

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
