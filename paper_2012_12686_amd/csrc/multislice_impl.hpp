// multislice_impl.hpp -- fused multislice forward / loss / adjoint kernels.
// Included by the instantiation units (one per probe size and split) and
// by the C ABI unit multislice.hip.
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
// object is read straight from HBM slice by slice.  Each position stores
// its contribution to the object gradient in its own staging planes (plain
// stores, no atomics); a second kernel sums the contributions of all
// positions for every voxel in position order, in FP64.  The reverse sweep
// rebuilds the wave
// entering each slice by stepping the forward recursion backwards
// (psi_{j-1} = t_{j-1}^{-1} P^H psi_j), and re-anchors it on checkpoints of
// the forward sweep stored every ckpt_every slices.  Where a checkpoint
// segment's transmissions absorb so strongly that dividing by them could
// amplify rounding by more than 2^4 (bounded per slice by a pre-pass over the
// object), the waves of that segment are instead recomputed forward from its
// checkpoint when the reverse sweep reaches it, kept in a per-position
// scratch area and read back like checkpoints.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "adorym.h"
#include "fastmath.hpp"
#include "tile.hpp"

using namespace adorym;

#include "context.hpp"

namespace adorym_ms {

struct MsParams {
  const float* a;          // delta or Re O, [S][Ly][Lx]
  const float* b;          // beta or Im O
  const float2* q;         // probe spectrum DFT(p)/N^2, natural [ky][kx]
  const int32_t* corner;   // [B][2]
  const float* shift;      // [B][2]
  const float* i_meas;     // [B][N][N]
  const float* i_total;    // [B][N][N] intensity summed over probe modes, or null (one mode)
  float* intensity;        // [B][N][N] or null
  float* g_a;              // [S][Ly][Lx] or null
  float* g_b;
  float* gstage;           // [B][S][2][N][N] per-position object-gradient contributions,
                           // null when no object gradient is wanted
  float2* ckpt;            // [B][nslots][K][R*THREADS]
  float2* recomp;          // [B][nrec][K][R*THREADS] waves of a recomputed segment
  float2* exit_wave;       // [B][K][R*THREADS] phi_{S-1} between the passes of a split evaluation
  float2* gacc;            // [B][N][N] natural, or null (probe-gradient partials)
  double* loss_part;       // [B][K]
  double* gs_part;         // [B][K][2] shift-gradient partials
  float2* xbuf;            // [B][2][2][N][N] exchange buffers (K > 1)
  int* counters;           // [B] group barrier counters (K > 1)
  int* xcc;                // [B][K] XCD ids of each group's members (K > 1)
  int* err;
  const double* gaps;      // [S-1] distance from slice j to j+1 (m): unequal spacing, or null
  const float2* nf_h;      // near field: [n_dist][N][N] transfer functions to the detector
  const float* nf_dph;     // near field: [N][N] d(phase of H)/d(distance), rad/m
  const int32_t* nf_idx;   // near field: [B] distance index of each position
  float2* nf_spec;         // near field: [B][K][R*THREADS] the detector spectrum H F phi (loss)
  double* nd_part;         // near field: [B][K] distance-gradient partials
  int n_dist;
  double* gd_part;         // [B][K][S-1] gap-gradient partials (unequal spacing)
  const float* absorb;     // [S] largest -log|t| of any voxel of each slice (absorb_bound_part)
  double chirp_per_m;      // lambda / dx^2: the Fresnel phase / pi of gap d is chirp_per_m d f^2
  int B, S, Ly, Lx, ckpt_every, nslots, nrec;
  int loss;                // ADORYM_LOSS_*
  int ksplit;              // workgroups per position of the launch that fills the partials
  float kdz;               // k * dz
  float adj_scale;         // multiplies the adjoint's seed, so every gradient (1: dL/d.)
  double chirp;            // lambda dz / dx^2
  double eps;
  double inv_n;            // 1 / (B N^2)
};

constexpr int kErrChunkRange = 1;   // error bit: a chunk left the object
constexpr int kErrDistIndex = 4;    // error bit: a distance index outside [0, n_dist)

__device__ __forceinline__ bool is_ckpt(int j, int S, int C) { return (j % C == 0) || (j == S - 1); }
__device__ __forceinline__ int ckpt_slot(int j, int S, int C) {
  return (j % C == 0) ? j / C : (S - 1) / C + 1;
}

// Inverse stepping through the checkpoint segment that starts at slice a
// divides the wave by t_i for every slice strictly between a and the next
// checkpoint, so rounding grows by at most exp(sum of the slices' largest
// -log|t|).  Past 2^4 (and for a transmission of zero, whose bound is
// infinite) the segment's waves are recomputed forward from its checkpoint.
constexpr float kMaxLogGain = 2.7725887f;   // log(16)

// The decisions of 64 consecutive segments (window `win`), one per lane,
// gathered by a ballot: bit i is segment 64 win + i.
__device__ __forceinline__ uint64_t seg_window_mask(const MsParams& P, int win) {
  const int a = (win * 64 + (int)(threadIdx.x & 63)) * P.ckpt_every;
  bool rc = false;
  if (P.absorb && a < P.S - 1) {
    const int e = min(a + P.ckpt_every, P.S - 1);
    float s = 0.f;
    for (int i = a + 1; i < e; ++i) s += P.absorb[i];
    rc = !(s <= kMaxLogGain);
  }
  return __ballot(rc);
}
// Segment decisions of the reverse sweep, computed one 64-segment window at
// a time (the sweep visits segments in decreasing order).  The segment of
// the last slice asked about is kept, so that consecutive slices of one
// segment cost two comparisons instead of integer divisions.
struct SegFlags {
  uint64_t mask = 0;
  int win = -1;
  int a = 1 << 30, e = 0;     // segment [a, e) of the last slice asked about
  bool rc = false;            // and whether it is recomputed
  __device__ __forceinline__ void locate(const MsParams& P, int j) {
    if (j >= a && j < e) return;
    a = j - j % P.ckpt_every;
    e = min(a + P.ckpt_every, P.S - 1);
    const int seg = a / P.ckpt_every;
    if ((seg >> 6) != win) {
      win = seg >> 6;
      mask = seg_window_mask(P, win);
    }
    rc = (mask >> (seg & 63)) & 1ull;
  }
  // slice j's segment is recomputed
  __device__ __forceinline__ bool recompute(const MsParams& P, int j) {
    locate(P, j);
    return rc;
  }
  // Slice j's entering wave is known exactly in the reverse sweep: stored,
  // or recomputed with the rest of its segment.
  __device__ __forceinline__ bool anchored(const MsParams& P, int j) {
    return is_ckpt(j, P.S, P.ckpt_every) || recompute(P, j);
  }
  // Slice j is the last slice of a segment to be recomputed: the reverse
  // sweep reaches that segment there.
  __device__ __forceinline__ bool entry(const MsParams& P, int j) {
    locate(P, j);
    return rc && j > a && j == e - 1;
  }
};

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
    const float att = exp_hw(-v), gain = __builtin_amdgcn_rcpf(att);
    t = make_float2(c * att, s * att);
    tinv = make_float2(c * gain, -s * gain);
  } else {
    t = make_float2(a, b);
    const float inv = 1.0f / (a * a + b * b);
    tinv = make_float2(a * inv, -b * inv);
  }
}

// Transmission of one slice on this thread's elements, computed ahead of
// its use: t, and for the reverse sweep g2 = |t|^-2 (t^-1 = conj(t) g2).
template <class C, int REPR, bool INV>
__device__ __forceinline__ void make_trans(float2 (&t)[C::R], float (&g2)[C::R], const float (&ca)[C::R],
                                           const float (&cb)[C::R], float kdz) {
  // phases within +-pi/4 on the whole wave (the usual case: k dz delta is a
  // few milliradians) skip the argument reduction
  bool small = true;
  if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
    float mx = 0.f;
#pragma unroll
    for (int m = 0; m < C::R; ++m) mx = fmaxf(mx, fabsf(kdz * ca[m]));
    small = __all(mx <= 0.78f);
  }
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
      float s, c;
      if (small) sincos_small_f32(kdz * ca[m], s, c);
      else sincos_f32(kdz * ca[m], s, c);
      const float v = kdz * cb[m];
      const float att = exp_hw(-v);
      t[m] = make_float2(c * att, s * att);
      if (INV) g2[m] = __builtin_amdgcn_rcpf(att * att);
    } else {
      t[m] = make_float2(ca[m], cb[m]);
      if (INV) g2[m] = 1.0f / (ca[m] * ca[m] + cb[m] * cb[m]);
    }
  }
}

// Shared memory of the multislice kernel.
template <class C>
struct MsShared {
  float2 buf[C::LDS_FIELD];   // transpose buffer (K == 1)
  Tables<C> tb;
  float2 ey[C::N];            // exp(-2 pi i s_y f(k)), natural k
  float2 ex[C::N];
  double red[2 * C::WAVES];
};

// Per-workgroup state: which field (position) and which part of it.
template <class C>
struct Work {
  Lane<C> ln;
  int b, part, cy, cx;
  Exchange x;
  SegFlags seg;
  __device__ __forceinline__ Work(int t, int b_, int part_) : ln(t, part_), b(b_), part(part_) {}
};

// Transpose one field / two fields (ROW <-> COL).
template <class C>
__device__ __forceinline__ void xfer(float2 (&v)[C::R], MsShared<C>& sh, Work<C>& wk, bool src_spec, bool dst_spec) {
  if constexpr (C::K == 1) transpose<C>(v, sh.buf, wk.ln, src_spec, dst_spec);
  else transpose_global<C, 1>(v, v, wk.x, wk.ln, src_spec, dst_spec);
}
template <class C>
__device__ __forceinline__ void xfer2(float2 (&v0)[C::R], float2 (&v1)[C::R], MsShared<C>& sh, Work<C>& wk,
                                      bool src_spec, bool dst_spec) {
  if constexpr (C::K == 1) {
    transpose<C>(v0, sh.buf, wk.ln, src_spec, dst_spec);
    transpose<C>(v1, sh.buf, wk.ln, src_spec, dst_spec);
  } else {
    transpose_global<C, 2>(v0, v1, wk.x, wk.ln, src_spec, dst_spec);
  }
}

// Fresnel propagation of one field along the thread's lines; the input is
// stashed in the thread's own cells of the LDS field buffer (or, for split
// fields with at most 8 values per lane, in registers, unless REGS is
// false).  K == 1 tiles share that buffer with the transposes, so they wait
// first: other waves may still be reading the row from the last transpose.
template <class C, bool CONJ, bool REGS = true>
__device__ __forceinline__ void prop(float2 (&v)[C::R], MsShared<C>& sh, const Lane<C>& ln) {
  // split fields with at most 8 values per lane keep the input in registers
  // (no LDS round trip; the register budget allows it except where the
  // unequal-spacing gradient already holds more live values)
  if constexpr (REGS && C::K > 1 && C::R <= 8) {
    propagate_line<C, CONJ>(v, sh.tb, ln);
    return;
  }
  if constexpr (C::K == 1) __syncthreads();
  propagate_line<C, CONJ>(v, sh.tb, ln, sh.buf + (ln.w * C::RPW + ln.g) * C::PITCH);
}

// Unequal slice spacing: the 1D Fresnel table of gap j, rebuilt in LDS
// before the propagations across that gap (in FP64, as the uniform table).
template <class C>
__device__ __forceinline__ void gap_table(MsShared<C>& sh, const MsParams& P, const Lane<C>& ln, int j) {
  __syncthreads();                           // every wave is done with the last table
  build_fresnel<C>(sh.tb, ln.tid, P.chirp_per_m * P.gaps[j]);
  __syncthreads();
}

// One axis of the gap gradient.  A gap d enters as psi' = F^-1[H F phi] with
// H = exp(i pi lambda d |nu|^2), and |nu|^2 splits into the two axes, so
// dL/dd = -(pi lambda / dx^2) Im sum conj(F lam') |f|^2 F psi' adds one
// term per axis; along an axis only the 1D transforms along it are needed
// (Parseval across the other axis), and the propagation along one axis
// leaves the term of the other axis unchanged.  Returns this thread's
// share of sum_k k^2 Im(conj(Lam_k) Psi_k) over its lines (unnormalised
// DFTs; the host applies -(pi lambda / dx^2) / N^3).
template <class C>
__device__ __forceinline__ float gap_term(const float2 (&psi)[C::R], const float2 (&lam)[C::R], const Tables<C>& tb,
                                          const Lane<C>& ln) {
  float2 x[C::R], y[C::R];
#pragma unroll
  for (int m = 0; m < C::R; ++m) { x[m] = psi[m]; y[m] = lam[m]; }
  fft_line<C, -1>(x, tb, ln);
  fft_line<C, -1>(y, tb, ln);
  float acc = 0.f;
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const int k = ln.pos_spec(m);
    const int kk = k < (C::N + 1) / 2 ? k : k - C::N;
    acc = fmaf(float(kk * kk), cmulc(x[m], y[m]).y, acc);   // k^2 Im(Psi conj(Lam))
  }
  return acc;
}

template <class C>
__device__ __forceinline__ void gap_store(const MsParams& P, MsShared<C>& sh, const Work<C>& wk, int gap, float acc) {
  const double t = block_sum<C::THREADS>((double)acc, sh.red);
  if (threadIdx.x == 0) P.gd_part[((size_t)wk.b * C::K + wk.part) * (P.S - 1) + gap] = t;
}

// Split-phase transposes of one (NF = 1) or two fields: xfer_begin ...
// independent work ... xfer_end.  K == 1 transposes through LDS at once.
template <class C, int NF>
__device__ __forceinline__ void xfer_begin(float2 (&v0)[C::R], float2 (&v1)[C::R], MsShared<C>& sh, Work<C>& wk,
                                           bool src_spec, bool dst_spec) {
  if constexpr (C::K == 1) {
    if constexpr (NF == 2) xfer2<C>(v0, v1, sh, wk, src_spec, dst_spec);
    else xfer<C>(v0, sh, wk, src_spec, dst_spec);
  } else {
    transpose_global_begin<C, NF>(v0, v1, wk.x, wk.ln, src_spec);
  }
}
template <class C, int NF>
__device__ __forceinline__ void xfer_end(float2 (&v0)[C::R], float2 (&v1)[C::R], Work<C>& wk, bool dst_spec) {
  if constexpr (C::K > 1) transpose_global_end<C, NF>(v0, v1, wk.x, wk.ln, dst_spec);
}

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

__device__ __forceinline__ rsrc_t slice_rsrc(const float* base, int j, const ChunkOffsets& o) {
  return make_rsrc(base + (size_t)j * (o.slice_bytes / 4), o.slice_bytes);
}

// This position's contribution to one object-gradient plane of slice j,
// chunk-local [N][N] (row y, column x).  Written once, read once by the
// reduction after the kernel.  Whole-field workgroups (K == 1) store it
// non-temporally (nt) so that it does not displace reused lines; split
// fields keep plain stores, whose partial lines the L2 combines (measured
// both ways).
template <class C>
__device__ __forceinline__ rsrc_t stage_rsrc(const MsParams& P, int b, int j, int comp) {
  constexpr int NN = C::N * C::N;
  return make_rsrc(P.gstage + (((size_t)b * P.S + j) * 2 + comp) * NN, NN * 4);
}
template <class C, bool ROW>
__device__ __forceinline__ void stage_store(rsrc_t r, const Lane<C>& ln, int m, float v) {
  constexpr int N = C::N;
  const uint32_t off = ROW ? (uint32_t)((ln.line * N + ln.q) * 4) : (uint32_t)((ln.q * N + ln.line) * 4);
  const uint32_t step = ROW ? 4 * C::L : 4 * C::L * N;
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off + (uint32_t)m * step, 0,
                                        C::K == 1 ? kNonTemporal : 0);
}

// Object values of slice j on this thread's elements (layout ROW/COL).
template <class C, bool ROW>
__device__ __forceinline__ void load_chunk(float (&ca)[C::R], float (&cb)[C::R], const MsParams& P,
                                           const ChunkOffsets& o, int j) {
  const rsrc_t ra = slice_rsrc(P.a, j, o), rb = slice_rsrc(P.b, j, o);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    ca[m] = chunk_load<C, ROW>(ra, o, m);
    cb[m] = chunk_load<C, ROW>(rb, o, m);
  }
}

// Modulate the wave by one slice (Eq. ri_modulation or complex_modulation).
template <class C, int REPR>
__device__ __forceinline__ void modulate(float2 (&v)[C::R], const float (&ca)[C::R], const float (&cb)[C::R],
                                         float kdz) {
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    float2 t, tinv;
    transmission<REPR>(kdz, ca[m], cb[m], t, tinv);
    v[m] = cmul(v[m], t);
  }
}

// Thread-native storage of this workgroup's part of a field.
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
__device__ __forceinline__ float2* ckpt_ptr(const MsParams& P, const Work<C>& wk, int slot) {
  return P.ckpt + (((size_t)wk.b * P.nslots + slot) * C::K + wk.part) * (C::R * C::THREADS);
}

// psi_0 = IDFT(Q e_b): Q loaded in COL layout (line kx, pos ky spectral).
template <class C>
__device__ __forceinline__ void place_probe(float2 (&v)[C::R], const MsParams& P, MsShared<C>& sh, Work<C>& wk) {
  const Lane<C>& ln = wk.ln;
  const float2 exv = sh.ex[ln.line];
  const rsrc_t rq = make_rsrc(P.q, C::N * C::N * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const int ky = ln.pos_spec(m);
    v[m] = cmul(bload2(rq, (uint32_t)(ky * C::N + ln.line) * 8, 0), cmul(sh.ey[ky], exv));
  }
  ifft_line<C, +1>(v, sh.tb, ln);                 // along y -> natural
  xfer<C>(v, sh, wk, false, true);                // -> ROW, x spectral
  ifft_line<C, +1>(v, sh.tb, ln);                 // along x -> natural
}

// One forward slice step of tiles that do not prefetch: (store) load the
// slice's object values, modulate, and propagate to slice j + 1.
template <class C, int REPR, bool ROW, bool CKPT, bool VAR = false>
__device__ __forceinline__ void forward_slice(float2 (&v)[C::R], float (&ca)[C::R], float (&cb)[C::R],
                                              const MsParams& P, MsShared<C>& sh, Work<C>& wk,
                                              const ChunkOffsets& o, int j) {
  if (CKPT && is_ckpt(j, P.S, P.ckpt_every)) field_store<C>(v, ckpt_ptr<C>(P, wk, ckpt_slot(j, P.S, P.ckpt_every)), wk.ln);
  load_chunk<C, ROW>(ca, cb, P, o, j);
  modulate<C, REPR>(v, ca, cb, P.kdz);
  if (j < P.S - 1) {
    if constexpr (VAR) gap_table<C>(sh, P, wk.ln, j);
    prop<C, false, !VAR>(v, sh, wk.ln);
    xfer<C>(v, sh, wk, false, false);
    prop<C, false, !VAR>(v, sh, wk.ln);
  }
}

template <class C>
__device__ __forceinline__ float2* recomp_ptr(const MsParams& P, const Work<C>& wk, int slot) {
  return P.recomp + (((size_t)wk.b * P.nrec + slot) * C::K + wk.part) * (C::R * C::THREADS);
}

// The waves entering slices a+1 .. e-1 of the segment that starts at the
// checkpoint of slice a (e: the next checkpoint), recomputed by the forward
// recursion with the same arithmetic as the forward sweep (tiles that
// prefetch modulate with make_trans, the others with modulate) and stored
// in the position's recompute slots; `v` is working storage.  The reverse
// sweep's other state (the adjoint field, a carried transmission) is not
// touched.
template <class C, int REPR, bool VAR>
__device__ __forceinline__ void recompute_segment(float2 (&v)[C::R], const MsParams& P, MsShared<C>& sh,
                                                  Work<C>& wk, const ChunkOffsets& o, int a) {
  const int e = min(a + P.ckpt_every, P.S - 1);
  field_load<C>(v, ckpt_ptr<C>(P, wk, ckpt_slot(a, P.S, P.ckpt_every)), wk.ln);
  for (int i = a; i < e - 1; ++i) {
    float ca[C::R], cb[C::R];
    if ((i & 1) == 0) load_chunk<C, true>(ca, cb, P, o, i);
    else load_chunk<C, false>(ca, cb, P, o, i);
    if constexpr (C::PREFETCH) {
      float2 t[C::R];
      float g2[C::R];
      make_trans<C, REPR, false>(t, g2, ca, cb, P.kdz);
#pragma unroll
      for (int m = 0; m < C::R; ++m) v[m] = cmul(v[m], t[m]);
    } else {
      modulate<C, REPR>(v, ca, cb, P.kdz);
    }
    if constexpr (VAR) gap_table<C>(sh, P, wk.ln, i);
    prop<C, false, !VAR>(v, sh, wk.ln);
    xfer<C>(v, sh, wk, false, false);
    prop<C, false, !VAR>(v, sh, wk.ln);
    field_store<C>(v, recomp_ptr<C>(P, wk, i - a), wk.ln);
  }
}

// Reverse slice step j (layout ROW/COL): gradient of slice j, then the two
// fields are taken back to slice j-1 by the adjoint propagator.
//   in : psi = phi_j (the wave leaving slice j, rebuilt by the backward
//        recursion) unless slice j is anchored on a checkpoint;
//        lam = dL/dphi_j
//   out: psi = phi_{j-1} = P^H psi_j, lam = dL/dphi_{j-1} = P^H conj(t_j) lam
// The slice gradient goes to this position's staging planes.  (Tiles that
// do not prefetch; backward_slice_pf below is the prefetching form.)
template <class C, int REPR, bool ROW, bool VAR = false>
__device__ __forceinline__ void backward_slice(float2 (&psi)[C::R], float2 (&lam)[C::R], float (&ca)[C::R],
                                               float (&cb)[C::R], const MsParams& P, MsShared<C>& sh, Work<C>& wk,
                                               const ChunkOffsets& o, int j) {
  const Lane<C>& ln = wk.ln;
  const bool stored = is_ckpt(j, P.S, P.ckpt_every);
  const bool anchored = stored || wk.seg.recompute(P, j);
  if (stored) field_load<C>(psi, ckpt_ptr<C>(P, wk, ckpt_slot(j, P.S, P.ckpt_every)), ln);  // psi_j exactly
  else if (anchored) field_load<C>(psi, recomp_ptr<C>(P, wk, j - wk.seg.a - 1), ln);   // recomputed
  load_chunk<C, ROW>(ca, cb, P, o, j);
  const bool grads = P.gstage != nullptr;
  const rsrc_t rga = grads ? stage_rsrc<C>(P, wk.b, j, 0) : make_rsrc(P.a, 0);
  const rsrc_t rgb = grads ? stage_rsrc<C>(P, wk.b, j, 1) : make_rsrc(P.b, 0);
  const float kdz = P.kdz;
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    float2 t, tinv;
    transmission<REPR>(kdz, ca[m], cb[m], t, tinv);
    const float2 in_wave = anchored ? psi[m] : cmul(psi[m], tinv);   // psi_j
    const float2 out_wave = anchored ? cmul(psi[m], t) : psi[m];     // phi_j
    const float2 l = lam[m];
    if (grads) {
      float ga, gb;
      if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
        const float2 z = cmulc(l, out_wave);          // lam conj(phi)
        ga = kdz * z.y;
        gb = -kdz * z.x;
      } else {
        const float2 z = cmulc(l, in_wave);           // lam conj(psi)
        ga = z.x;
        gb = z.y;
      }
      stage_store<C, ROW>(rga, ln, m, ga);
      stage_store<C, ROW>(rgb, ln, m, gb);
    }
    lam[m] = cmulc(l, t);                              // conj(t) lam = dL/dpsi_j
    psi[m] = in_wave;
  }
  if (j > 0) {
    // unequal spacing: the gap gradient needs psi across the gap every time
    const bool need_psi = VAR || !wk.seg.anchored(P, j - 1);
    if (need_psi) {
      float gacc = 0.f;
      if constexpr (VAR) {
        gap_table<C>(sh, P, ln, j - 1);
        gacc = gap_term<C>(psi, lam, sh.tb, ln);
      }
      prop<C, true, !VAR>(psi, sh, ln);
      prop<C, true, !VAR>(lam, sh, ln);
      xfer2<C>(psi, lam, sh, wk, false, false);
      if constexpr (VAR) gacc += gap_term<C>(psi, lam, sh.tb, ln);
      prop<C, true, !VAR>(psi, sh, ln);
      prop<C, true, !VAR>(lam, sh, ln);
      if constexpr (VAR) gap_store<C>(P, sh, wk, j - 1, gacc);
    } else {
      prop<C, true, !VAR>(lam, sh, ln);
      xfer<C>(lam, sh, wk, false, false);
      prop<C, true, !VAR>(lam, sh, ln);
    }
  }
}

// Slice steps of tiles that prefetch (C::PREFETCH): the object values of
// the next slice are loaded during the propagation, and its transmission is
// computed while the transpose's exchange is in flight (between the two
// halves of the split barrier).  t/g2 carry the transmission of the current
// slice from step to step.
template <class C, int REPR, bool ROW, bool CKPT, bool VAR = false>
__device__ __forceinline__ void forward_slice_pf(float2 (&v)[C::R], float2 (&t)[C::R], float (&g2)[C::R],
                                                 const MsParams& P, MsShared<C>& sh, Work<C>& wk,
                                                 const ChunkOffsets& o, int j) {
  if (CKPT && is_ckpt(j, P.S, P.ckpt_every)) field_store<C>(v, ckpt_ptr<C>(P, wk, ckpt_slot(j, P.S, P.ckpt_every)), wk.ln);
#pragma unroll
  for (int m = 0; m < C::R; ++m) v[m] = cmul(v[m], t[m]);
  if (j < P.S - 1) {
    if constexpr (VAR) gap_table<C>(sh, P, wk.ln, j);
    float ca[C::R], cb[C::R];
    load_chunk<C, !ROW>(ca, cb, P, o, j + 1);   // in flight during the propagation
    prop<C, false, !VAR>(v, sh, wk.ln);
    xfer_begin<C, 1>(v, v, sh, wk, false, false);
    make_trans<C, REPR, false>(t, g2, ca, cb, P.kdz);
    xfer_end<C, 1>(v, v, wk, false);
    prop<C, false, !VAR>(v, sh, wk.ln);
  }
}

template <class C, int REPR, bool ROW, bool VAR = false>
__device__ __forceinline__ void backward_slice_pf(float2 (&psi)[C::R], float2 (&lam)[C::R], float2 (&t)[C::R],
                                                  float (&g2)[C::R], const MsParams& P, MsShared<C>& sh,
                                                  Work<C>& wk, const ChunkOffsets& o, int j) {
  const Lane<C>& ln = wk.ln;
  const bool stored = is_ckpt(j, P.S, P.ckpt_every);
  const bool anchored = stored || wk.seg.recompute(P, j);
  if (stored) field_load<C>(psi, ckpt_ptr<C>(P, wk, ckpt_slot(j, P.S, P.ckpt_every)), ln);  // psi_j exactly
  else if (anchored) field_load<C>(psi, recomp_ptr<C>(P, wk, j - wk.seg.a - 1), ln);   // recomputed
  const bool grads = P.gstage != nullptr;
  const rsrc_t rga = grads ? stage_rsrc<C>(P, wk.b, j, 0) : make_rsrc(P.a, 0);
  const rsrc_t rgb = grads ? stage_rsrc<C>(P, wk.b, j, 1) : make_rsrc(P.b, 0);
  const float kdz = P.kdz;
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const float2 tm = t[m];
    const float2 in_wave = anchored ? psi[m] : cscale(cmulc(psi[m], tm), g2[m]);   // psi_j = phi_j / t_j
    const float2 out_wave = anchored ? cmul(psi[m], tm) : psi[m];                  // phi_j
    const float2 l = lam[m];
    if (grads) {
      float ga, gb;
      if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
        const float2 z = cmulc(l, out_wave);          // lam conj(phi)
        ga = kdz * z.y;
        gb = -kdz * z.x;
      } else {
        const float2 z = cmulc(l, in_wave);           // lam conj(psi)
        ga = z.x;
        gb = z.y;
      }
      stage_store<C, ROW>(rga, ln, m, ga);
      stage_store<C, ROW>(rgb, ln, m, gb);
    }
    lam[m] = cmulc(l, tm);                             // conj(t) lam = dL/dpsi_j
    psi[m] = in_wave;
  }
  if (j > 0) {
    float gacc = 0.f;
    if constexpr (VAR) {
      gap_table<C>(sh, P, ln, j - 1);
      gacc = gap_term<C>(psi, lam, sh.tb, ln);
    }
    float ca[C::R], cb[C::R];
    load_chunk<C, !ROW>(ca, cb, P, o, j - 1);   // in flight during the propagation
    // unequal spacing: the gap gradient needs psi across the gap every time
    const bool need_psi = VAR || !wk.seg.anchored(P, j - 1);
    if (need_psi) {
      prop<C, true, !VAR>(psi, sh, ln);
      prop<C, true, !VAR>(lam, sh, ln);
      xfer_begin<C, 2>(psi, lam, sh, wk, false, false);
      make_trans<C, REPR, true>(t, g2, ca, cb, kdz);
      xfer_end<C, 2>(psi, lam, wk, false);
      if constexpr (VAR) gacc += gap_term<C>(psi, lam, sh.tb, ln);
      prop<C, true, !VAR>(psi, sh, ln);
      prop<C, true, !VAR>(lam, sh, ln);
      if constexpr (VAR) gap_store<C>(P, sh, wk, j - 1, gacc);
    } else {
      prop<C, true, !VAR>(lam, sh, ln);
      xfer_begin<C, 1>(lam, lam, sh, wk, false, false);
      make_trans<C, REPR, true>(t, g2, ca, cb, kdz);
      xfer_end<C, 1>(lam, lam, wk, false);
      prop<C, true, !VAR>(lam, sh, ln);
    }
  }
}

// Map the workgroup index to (position, part).  The K parts of a position
// sit in consecutive slots of one XCD (workgroups are dealt to the 8 XCDs
// round-robin), so their exchange traffic stays in that XCD's L2.
template <class C>
__device__ __forceinline__ void group_of_block(int& b, int& part) {
  const int i = blockIdx.x;
  const int xcd = i & 7, slot = i >> 3;
  b = (slot / C::K) * 8 + xcd;
  part = slot % C::K;
}

// Everything one workgroup does for its part of one position.  wk.b, wk.part
// and the exchange state wk.x are set by the caller.
// Near field: the 2D transfer function to the detector between a DFT and
// an inverse DFT over both axes.  In : the wave in the layout of slice S-1,
// natural order.  Out: the propagated wave in the same layout, natural
// order, times N^2 (unnormalised transforms).  CONJ applies conj(H) (the
// adjoint); `stash`, if given, receives H F v (thread-native order) and,
// with `dz`, the distance-gradient term sum dph Im((F v) conj(stash)) is
// accumulated into *dz.
template <class C, bool CONJ>
__device__ __forceinline__ void nearfield_prop(float2 (&v)[C::R], const float2* __restrict__ h,
                                               const float* __restrict__ dph, MsShared<C>& sh, Work<C>& wk,
                                               float2* stash_out, const float2* stash_in, float* dz) {
  const Lane<C>& ln = wk.ln;
  constexpr int N = C::N;
  fft_line<C, -1>(v, sh.tb, ln);
  xfer<C>(v, sh, wk, true, false);
  fft_line<C, -1>(v, sh.tb, ln);
  // element m: line = one axis's frequency (natural index), pos_spec(m) = the other's;
  // H depends on |nu|^2 only, so its table is symmetric
  float acc = 0.f;
  float2 st[C::R];
  if (stash_in) {
    const rsrc_t r = make_rsrc(stash_in, C::R * C::THREADS * 8);
#pragma unroll
    for (int m = 0; m < C::R; ++m) st[m] = bload2(r, ln.tid * 8, m * C::THREADS * 8);
  }
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const int idx = ln.line * N + ln.pos_spec(m);
    if (stash_in) acc = fmaf(dph[idx], cmulc(v[m], st[m]).y, acc);
    const float2 hv = h[idx];
    v[m] = CONJ ? cmulc(v[m], hv) : cmul(v[m], hv);
  }
  if (dz) *dz = acc;
  if (stash_out) field_store<C>(v, stash_out, ln);
  ifft_line<C, +1>(v, sh.tb, ln);
  xfer<C>(v, sh, wk, false, true);
  ifft_line<C, +1>(v, sh.tb, ln);
}

// SPLIT: the evaluation in two launches (several probe modes, whose loss
// needs every mode's intensity first).  The forward launch (LOSS false)
// stores the checkpoints and the exit wave; the loss launch resumes from
// them instead of repeating the forward sweep.
template <class C, int REPR, bool LOSS, bool VAR = false, bool NF = false, bool SPLIT = false>
__device__ __forceinline__ void process_position(const MsParams& P, MsShared<C>& sh, Work<C>& wk) {
  const int b = wk.b, part = wk.part;
  const Lane<C>& ln = wk.ln;
  constexpr int N = C::N;
  constexpr int NN = N * N;
  wk.seg = SegFlags();                        // decisions belong to this job's object
  wk.cy = P.corner[2 * b];
  wk.cx = P.corner[2 * b + 1];
  const float sy = P.shift[2 * b], sx = P.shift[2 * b + 1];

  // TakeObjectChunk: the chunk must lie inside the object (and a near-field
  // position's distance index inside the distance list).
  const int didx = NF ? P.nf_idx[b] : 0;
  const bool bad_dist = NF && (didx < 0 || didx >= P.n_dist);
  if (wk.cy < 0 || wk.cx < 0 || wk.cy + N > P.Ly || wk.cx + N > P.Lx || bad_dist) {
    if (threadIdx.x == 0 && part == 0) atomicOr(P.err, bad_dist ? kErrDistIndex : kErrChunkRange);
    if (LOSS) {
      if (threadIdx.x == 0) {
        P.loss_part[b * C::K + part] = 0.0;
        P.gs_part[2 * (b * C::K + part)] = 0.0;
        P.gs_part[2 * (b * C::K + part) + 1] = 0.0;
      }
      if (P.gacc)
        for (int i = part * C::THREADS + threadIdx.x; i < NN; i += C::K * C::THREADS)
          P.gacc[(size_t)b * NN + i] = make_float2(0.f, 0.f);
      if (VAR)
        for (int i = threadIdx.x; i < P.S - 1; i += C::THREADS)
          P.gd_part[((size_t)b * C::K + part) * (P.S - 1) + i] = 0.0;
      if (NF && threadIdx.x == 0) P.nd_part[b * C::K + part] = 0.0;
    }
    if (P.intensity)
      for (int i = part * C::THREADS + threadIdx.x; i < NN; i += C::K * C::THREADS)
        P.intensity[(size_t)b * NN + i] = 0.f;
    return;
  }

  setup_tables<C>(sh, ln, P.chirp, sy, sx);
  const ChunkOffsets o = chunk_offsets<C>(ln, wk.cy, wk.cx, P.Ly, P.Lx);

  float2 v[C::R];
  // object values of the current slice (tiles that do not prefetch), or the
  // current slice's transmission (tiles that do)
  float ca[C::R], cb[C::R];
  float2 tr[C::R];
  float g2[C::R];
  const bool last_row = ((P.S - 1) & 1) == 0;
  float2* const exit_slot = SPLIT ? P.exit_wave + ((size_t)b * C::K + part) * (C::R * C::THREADS) : nullptr;
  constexpr bool CKPT = LOSS || SPLIT;
  if constexpr (SPLIT && LOSS) {
    // resume: the exit wave and the checkpoints of this position are stored
    field_load<C>(v, exit_slot, ln);
    if constexpr (C::PREFETCH) {
#pragma unroll
      for (int m = 0; m < C::R; ++m) g2[m] = 1.0f;
      if (last_row) load_chunk<C, true>(ca, cb, P, o, P.S - 1);
      else load_chunk<C, false>(ca, cb, P, o, P.S - 1);
      make_trans<C, REPR, false>(tr, g2, ca, cb, P.kdz);
    }
  } else {
    if constexpr (C::PREFETCH) {
      load_chunk<C, true>(ca, cb, P, o, 0);
#pragma unroll
      for (int m = 0; m < C::R; ++m) g2[m] = 1.0f;   // slice S-1 is always anchored: no inverse needed
      make_trans<C, REPR, false>(tr, g2, ca, cb, P.kdz);
    }
    place_probe<C>(v, P, sh, wk);

    // MultislicePropagate: even slices in ROW layout, odd slices in COL layout.
    for (int j = 0; j < P.S; j += 2) {
      if constexpr (C::PREFETCH) {
        forward_slice_pf<C, REPR, true, CKPT, VAR>(v, tr, g2, P, sh, wk, o, j);
        if (j + 1 < P.S) forward_slice_pf<C, REPR, false, CKPT, VAR>(v, tr, g2, P, sh, wk, o, j + 1);
      } else {
        forward_slice<C, REPR, true, CKPT, VAR>(v, ca, cb, P, sh, wk, o, j);
        if (j + 1 < P.S) forward_slice<C, REPR, false, CKPT, VAR>(v, ca, cb, P, sh, wk, o, j + 1);
      }
    }
    if constexpr (SPLIT) field_store<C>(v, exit_slot, ln);
  }

  float2* nf_slot = nullptr;
  if constexpr (NF) {
    // Fresnel propagation to the detector: natural order in the layout of slice S-1
    nf_slot = P.nf_spec + ((size_t)b * C::K + part) * (C::R * C::THREADS);
    nearfield_prop<C, false>(v, P.nf_h + (size_t)didx * NN, P.nf_dph, sh, wk, LOSS ? nf_slot : nullptr, nullptr,
                             nullptr);
  } else {
    // FarFieldPropagate: inverse DFT along the current lines, transpose, along
    // the other axis.  Result: spectral along the lines of the final layout.
    fft_line<C, +1>(v, sh.tb, ln);
    xfer<C>(v, sh, wk, true, false);
    fft_line<C, +1>(v, sh.tb, ln);
  }
  const float inv_nf = NF ? 1.0f / float(NN) : 1.0f / float(N);

  // Per-pixel loss terms in FP32; the sum over pixels is accumulated in FP64.
  double lsum = 0.0;
  const float eps = (float)P.eps;
  const float inv_n = (float)P.inv_n;
  const rsrc_t rim = make_rsrc(LOSS ? (const void*)(P.i_meas + (size_t)b * NN) : (const void*)P.q, NN * 4);
  const rsrc_t rtot = make_rsrc(P.i_total ? (const void*)(P.i_total + (size_t)b * NN) : (const void*)P.q, NN * 4);
  const rsrc_t rint = make_rsrc(P.intensity ? (const void*)(P.intensity + (size_t)b * NN) : (const void*)P.q, NN * 4);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    int ky, kx;
    uint32_t det;
    if constexpr (NF) {
      // natural order in the layout of slice S-1: ROW when S-1 is even
      if (last_row) { ky = ln.line; kx = ln.pos_nat(m); }
      else          { ky = ln.pos_nat(m); kx = ln.line; }
      det = (uint32_t)(ky * N + kx) * 4;
    } else {
      if (last_row) { ky = ln.pos_spec(m); kx = ln.line; }    // final layout COL
      else          { ky = ln.line; kx = ln.pos_spec(m); }    // final layout ROW
      det = (uint32_t)(((ky + N / 2) % N) * N + (kx + N / 2) % N) * 4;
    }
    const float2 psi_det = cscale(v[m], inv_nf);
    const float ip = psi_det.x * psi_det.x + psi_det.y * psi_det.y;
    if (P.intensity) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, ip), rint, det, 0, 0);
    if (LOSS) {
      const float imv = bload(rim, det, 0);
      // the loss is a function of the detector intensity: with several probe
      // modes that is their sum (Eq. multimode), this mode's own otherwise
      const float it = P.i_total ? bload(rtot, det, 0) : ip;
      float term, dldi;
      if (P.loss == ADORYM_LOSS_GAUSSIAN) {
        const float sp = sqrtf(it + eps), sm = sqrtf(imv + eps);
        term = (sp - sm) * (sp - sm);
        dldi = (1.0f - sm / sp) * inv_n;
      } else {
        term = it - imv * logf(it + eps);
        dldi = (1.0f - imv / (it + eps)) * inv_n;
      }
      lsum += (double)term;
      // far-field residual 2 dL/dI Psi, scaled by 1/N for the adjoint DFT
      v[m] = cscale(psi_det, 2.0f * dldi * (inv_nf * P.adj_scale));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (!LOSS) return;

  {
    double tot = block_sum<C::THREADS>(lsum, sh.red);
    if (threadIdx.x == 0) P.loss_part[b * C::K + part] = tot * P.inv_n;   // mean over the B N^2 pixels
  }

  if constexpr (NF) {
    // Adjoint of the detector propagation (conj(H)), and the distance
    // gradient from the stashed spectrum
    float dz = 0.f;
    nearfield_prop<C, true>(v, P.nf_h + (size_t)didx * NN, P.nf_dph, sh, wk, nullptr, nf_slot, &dz);
    const double tz = block_sum<C::THREADS>((double)dz, sh.red);
    if (threadIdx.x == 0) P.nd_part[b * C::K + part] = tz;
  } else {
    // Adjoint of the far field: DFT back along the two axes.
    ifft_line<C, -1>(v, sh.tb, ln);
    xfer<C>(v, sh, wk, false, true);
    ifft_line<C, -1>(v, sh.tb, ln);
  }
  // v = lambda_{S-1} in the layout of slice S-1

  float2 psi[C::R];
  int j = P.S - 1;
  // the forward sweep left slice S-1's object values in ca/cb (or its
  // transmission in tr)
  if constexpr (C::PREFETCH) {
    if (!last_row) {
      backward_slice_pf<C, REPR, false, VAR>(psi, v, tr, g2, P, sh, wk, o, j);
      --j;
    }
    for (; j >= 1; j -= 2) {
      // a segment to recompute is reached at j or j - 1 (slice j is then its
      // checkpoint or its last slice, so psi is free)
      if (wk.seg.entry(P, j) || wk.seg.entry(P, j - 1)) recompute_segment<C, REPR, VAR>(psi, P, sh, wk, o, wk.seg.a);
      backward_slice_pf<C, REPR, true, VAR>(psi, v, tr, g2, P, sh, wk, o, j);
      backward_slice_pf<C, REPR, false, VAR>(psi, v, tr, g2, P, sh, wk, o, j - 1);
    }
    if (j == 0) backward_slice_pf<C, REPR, true, VAR>(psi, v, tr, g2, P, sh, wk, o, 0);
  } else {
    if (!last_row) {
      backward_slice<C, REPR, false, VAR>(psi, v, ca, cb, P, sh, wk, o, j);
      --j;
    }
    // now slice j is even (ROW); pairs (j ROW, j-1 COL) down to slice 0
    for (; j >= 1; j -= 2) {
      if (wk.seg.entry(P, j) || wk.seg.entry(P, j - 1)) recompute_segment<C, REPR, VAR>(psi, P, sh, wk, o, wk.seg.a);
      backward_slice<C, REPR, true, VAR>(psi, v, ca, cb, P, sh, wk, o, j);
      backward_slice<C, REPR, false, VAR>(psi, v, ca, cb, P, sh, wk, o, j - 1);
    }
    if (j == 0) backward_slice<C, REPR, true, VAR>(psi, v, ca, cb, P, sh, wk, o, 0);
  }
  // v = dL/d(shifted probe) in ROW layout, natural order.

  // FourierShift adjoint: G = DFT(g_pb) in COL layout (kx line, ky spectral).
  fft_line<C, -1>(v, sh.tb, ln);
  xfer<C>(v, sh, wk, true, false);
  fft_line<C, -1>(v, sh.tb, ln);
  const float2 exv = sh.ex[ln.line];
  const double fx = freq<N>(ln.line);
  double gsy = 0.0, gsx = 0.0;
  const rsrc_t rq = make_rsrc(P.q, NN * 8);
  const rsrc_t rg = make_rsrc(P.gacc ? P.gacc + (size_t)b * NN : P.q, NN * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const int ky = ln.pos_spec(m);
    const uint32_t off = (uint32_t)(ky * N + ln.line) * 8;
    const float2 e = cmul(sh.ey[ky], exv);
    const float2 g = v[m];
    if (P.gacc) bstore2(rg, cmulc(g, e), off, 0);
    const float2 qv = bload2(rq, off, 0);
    const float2 z = cmul(cmulc(qv, g), e);     // conj(G) Q e
    gsy += freq<N>(ky) * double(z.y);
    gsx += fx * double(z.y);
  }
  double ty = block_sum<C::THREADS>(gsy, sh.red);
  double tx = block_sum<C::THREADS>(gsx, sh.red + C::WAVES);
  if (threadIdx.x == 0) {
    const double two_pi = 6.283185307179586476925286766559;
    P.gs_part[2 * (b * C::K + part)] = two_pi * ty;
    P.gs_part[2 * (b * C::K + part) + 1] = two_pi * tx;
  }
}

// One group of K workgroups per position of a single job.
template <class C, int REPR, bool LOSS, bool VAR = false, bool NF = false, bool SPLIT = false>
__global__ void __launch_bounds__(C::THREADS) multislice_kernel(MsParams P) {
  __shared__ MsShared<C> sh;
  int b, part;
  group_of_block<C>(b, part);
  if (b >= P.B) return;                       // padding of the XCD-aware grid
  Work<C> wk(threadIdx.x, b, part);
  wk.x.buf = P.xbuf + (size_t)b * 4 * C::N * C::N;
  wk.x.counter = P.counters + b;
  wk.x.err = P.err;
  wk.x.phase = 0;
  wk.x.local = false;
  const int cy = P.corner[2 * b], cx = P.corner[2 * b + 1];
  const bool inside = cy >= 0 && cx >= 0 && cy + C::N <= P.Ly && cx + C::N <= P.Lx;
  if (C::K > 1 && inside) exchange_init<C::K>(wk.x, P.xcc + b * C::K, part);
  process_position<C, REPR, LOSS, VAR, NF, SPLIT>(P, sh, wk);
}

// Persistent multi-job kernel: groups of K workgroups take (job, position)
// items from a device queue until it is empty.  Every member of a group sees
// the same ticket (member 0 draws it and publishes it behind the group
// barrier), so all of them leave the loop together.
template <class C, int REPR>
__global__ void __launch_bounds__(C::THREADS) multislice_batched_kernel(const MsParams* __restrict__ jobs,
                                                                        const int2* __restrict__ items,
                                                                        int n_items, int* ticket, int* mailbox,
                                                                        int* counters, int* xcc, float2* xbuf,
                                                                        int* err) {
  __shared__ MsShared<C> sh;
  __shared__ int sh_ticket;
  int g, part;
  group_of_block<C>(g, part);
  Work<C> wk(threadIdx.x, 0, part);
  wk.x.buf = xbuf + (size_t)g * 4 * C::N * C::N;
  wk.x.counter = counters + g;
  wk.x.err = err;
  wk.x.phase = 0;
  wk.x.local = false;
  if (C::K > 1) exchange_init<C::K>(wk.x, xcc + g * C::K, part);
  for (;;) {
    int t;
    if constexpr (C::K == 1) {
      __syncthreads();
      if (threadIdx.x == 0) sh_ticket = atomicAdd(ticket, 1);
      __syncthreads();
      t = sh_ticket;
    } else {
      if (threadIdx.x == 0 && part == 0)
        __hip_atomic_store(mailbox + g, atomicAdd(ticket, 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ++wk.x.phase;
      group_barrier(wk.x.counter, C::K * wk.x.phase, wk.x.err);
      t = __hip_atomic_load(mailbox + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the ticket is the same for the whole workgroup: make that visible so
    // the item and the job's parameters are loaded into scalar registers
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= n_items) break;
    const int2 it = items[t];
    wk.b = __builtin_amdgcn_readfirstlane(it.y);
    process_position<C, REPR, true>(jobs[__builtin_amdgcn_readfirstlane(it.x)], sh, wk);
  }
}

// Probe defocus (a refinable parameter of the experiment, Sec. S1.D): the
// probe is Fresnel-propagated (Eqs. fresnel_prop, paraxial_kernel) by a
// distance d before it meets the object, i.e. its spectrum is multiplied by
// H(nu) = exp(i pi lambda d |nu|^2).  `c0` is pi lambda / (N dx)^2, so the
// phase at natural-order frequency (ky, kx) is c0 d (fy^2 + fx^2) with
// fy = ky or ky - N (NumPy's fftfreq order).  Built in FP64, rounded once.
struct Defocus {
  double dist;       // metres
  double c0;         // pi lambda / (N dx)^2, 1/m
  double* g_dist;    // device FP64 scalar, or NULL
};

__device__ __forceinline__ double defocus_nu2(int i, int n) {
  const int ky = i / n, kx = i - ky * n;
  const double fy = ky < n / 2 ? ky : ky - n, fx = kx < n / 2 ? kx : kx - n;
  return fy * fy + fx * fx;
}

// q <- q H, in place (the spectrum the multislice kernel places).
static __global__ void __launch_bounds__(256) defocus_spectrum_kernel(float2* __restrict__ q, int n, double c0,
                                                                      double dist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  double sn, cs;
  sincos(c0 * dist * defocus_nu2(i, n), &sn, &cs);
  q[i] = cmul(q[i], make_float2((float)cs, (float)sn));
}

// Before the probe-gradient transform: with G = dL/dq_d (the per-position sum,
// natural order) and q_d = q H, dL/dd = Re sum conj(G) (i c0 nu2) q_d
// = -sum c0 nu2 Im(conj(G) q_d); then G <- conj(H) G, the gradient with
// respect to the undefocused spectrum.  kDefocusParts workgroups each sum a
// fixed contiguous share (strided per thread, then a tree) into `part`;
// defocus_finish_kernel adds the shares in order: FP64, bitwise reproducible.
constexpr int kDefocusParts = 64;
static __global__ void __launch_bounds__(256) defocus_grad_kernel(float2* __restrict__ g, const float2* __restrict__ qd,
                                                                  int n, double c0, double dist,
                                                                  double* __restrict__ part) {
  __shared__ double red[256];
  const int share = (n * n + kDefocusParts - 1) / kDefocusParts;
  const int lo = blockIdx.x * share, hi = min(n * n, lo + share);
  double s = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double nu2 = defocus_nu2(i, n);
    const float2 gi = g[i], qi = qd[i];
    s -= c0 * nu2 * ((double)gi.x * qi.y - (double)gi.y * qi.x);
    double sn, cs;
    sincos(c0 * dist * nu2, &sn, &cs);
    g[i] = cmulc(gi, make_float2((float)cs, (float)sn));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
static __global__ void __launch_bounds__(kDefocusParts) defocus_finish_kernel(const double* __restrict__ part,
                                                                              double* __restrict__ g_dist,
                                                                              int accumulate) {
  __shared__ double red[kDefocusParts];
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int h = kDefocusParts / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && g_dist) *g_dist = accumulate ? *g_dist + red[0] : red[0];
}

// Grid of the one-group probe kernels.  Workgroups are dealt to the eight
// XCDs in turn, so with K > 1 the grid holds 8 K workgroups and only every
// eighth works (part = index / 8): the K members then share one XCD and
// exchange through its L2 (exchange_init checks this; members on several
// XCDs would still exchange correctly, through memory).
template <class C>
constexpr unsigned probe_grid() { return C::K > 1 ? 8u * C::K : 1u; }
template <class C>
__device__ __forceinline__ int probe_part() { return C::K > 1 ? (int)(blockIdx.x >> 3) : 0; }
template <class C>
__device__ __forceinline__ bool probe_idle() { return C::K > 1 && (blockIdx.x & 7) != 0; }

static __global__ void reset_ints_kernel(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Per slice j, the largest -log|t| over the slice's voxels, i.e. the most a
// division by t_j can amplify a value (log scale; negative values count as
// 0): k dz beta for delta/beta objects, -log|O| for real/imaginary ones
// (infinite where O = 0).  Each of `parts` workgroups of a slice takes one
// strided share of its voxels; non-negative floats order like their bit
// patterns, so the shares combine by an integer maximum into out[j]
// (cleared before).  NaN voxels are ignored.
template <int REPR>
__device__ __forceinline__ float absorb_gain(float kdz, float x, float y) {
  if constexpr (REPR == ADORYM_OBJ_DELTA_BETA) {
    return kdz * y;
  } else {
    const float m2 = x * x + y * y;
    return m2 > 0.f ? -0.5f * logf(m2) : INFINITY;
  }
}
template <int REPR, int THREADS>
__device__ void absorb_bound_part(const float* __restrict__ a, const float* __restrict__ b, size_t plane, float kdz,
                                  unsigned* __restrict__ out, int j, int part, int parts, float* wmax) {
  const float* pa = a + (size_t)j * plane;
  const float* pb = b + (size_t)j * plane;
  float mx = 0.f;
  const size_t stride = (size_t)parts * THREADS;
  if ((plane & 3) == 0 && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0) {
    // four voxels per load (every slice starts on a 16-byte boundary)
    const float4* qa = reinterpret_cast<const float4*>(pa);
    const float4* qb = reinterpret_cast<const float4*>(pb);
    for (size_t i = (size_t)part * THREADS + threadIdx.x; i < plane / 4; i += stride) {
      const float4 y = qb[i];
      const float4 x = REPR == ADORYM_OBJ_DELTA_BETA ? y : qa[i];
      mx = fmaxf(mx, fmaxf(fmaxf(absorb_gain<REPR>(kdz, x.x, y.x), absorb_gain<REPR>(kdz, x.y, y.y)),
                           fmaxf(absorb_gain<REPR>(kdz, x.z, y.z), absorb_gain<REPR>(kdz, x.w, y.w))));
    }
  } else {
    for (size_t i = (size_t)part * THREADS + threadIdx.x; i < plane; i += stride)
      mx = fmaxf(mx, absorb_gain<REPR>(kdz, REPR == ADORYM_OBJ_DELTA_BETA ? 0.f : pa[i], pb[i]));
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (int w = 0; w < THREADS / 64; ++w) m = fmaxf(m, wmax[w]);
    atomicMax(out + j, __float_as_uint(m));
  }
}

// The per-slice absorption bounds of one object, computed by workgroups of
// the probe-spectrum launch (null `out`: none).
struct AbsorbJob {
  const float* a;
  const float* b;
  size_t plane;             // voxels per slice
  float kdz;
  unsigned* out;            // [S], cleared before the launch
  int parts;                // workgroups per slice
  int repr;                 // ADORYM_OBJ_*
};

// Probe spectrum Q = DFT(p) / N^2 (natural [ky][kx]).  One group of K
// workgroups (probe_grid); K > 1 exchanges through xbuf.  The workgroups
// after the group's grid compute the absorption bounds of `ab`, parts
// workgroups per slice (they need nothing from the spectrum).
template <class C>
__global__ void __launch_bounds__(C::THREADS) probe_spectrum_kernel(const float2* __restrict__ probe,
                                                                    float2* __restrict__ q, float2* xbuf,
                                                                    int* counter, int* xcc, int* err,
                                                                    AbsorbJob ab) {
  __shared__ MsShared<C> sh;
  if (blockIdx.x >= probe_grid<C>()) {
    const int i = (int)(blockIdx.x - probe_grid<C>());
    float* wmax = reinterpret_cast<float*>(sh.red);
    if (ab.repr == ADORYM_OBJ_DELTA_BETA)
      absorb_bound_part<ADORYM_OBJ_DELTA_BETA, C::THREADS>(ab.a, ab.b, ab.plane, ab.kdz, ab.out, i / ab.parts,
                                                            i % ab.parts, ab.parts, wmax);
    else
      absorb_bound_part<ADORYM_OBJ_REAL_IMAG, C::THREADS>(ab.a, ab.b, ab.plane, ab.kdz, ab.out, i / ab.parts,
                                                           i % ab.parts, ab.parts, wmax);
    return;
  }
  if (probe_idle<C>()) return;
  const int part = probe_part<C>();
  Work<C> wk(threadIdx.x, 0, part);
  wk.x.buf = xbuf; wk.x.counter = counter; wk.x.err = err; wk.x.phase = 0; wk.x.local = false;
  const Lane<C>& ln = wk.ln;
  build_twiddles<C>(sh.tb, ln.tid);
  __syncthreads();
  if constexpr (C::K > 1) exchange_init<C::K>(wk.x, xcc, part);
  constexpr int N = C::N;
  float2 v[C::R];
#pragma unroll
  for (int m = 0; m < C::R; ++m) v[m] = probe[ln.line * N + ln.pos_nat(m)];
  fft_line<C, -1>(v, sh.tb, ln);
  xfer<C>(v, sh, wk, true, false);
  fft_line<C, -1>(v, sh.tb, ln);
  const float s = 1.0f / float(N * N);
#pragma unroll
  for (int m = 0; m < C::R; ++m) q[ln.pos_spec(m) * N + ln.line] = cscale(v[m], s);
}


// Sums of the per-position partials: probe-gradient spectrum (natural
// order, positions in index order; workgroup `blk` of `nblk` takes every
// nblk-th run of 256 elements), loss (workgroup 0: a fixed-order strided sum
// per thread, then a fixed-order tree), shift gradients (workgroup 0).
// 256 threads; `red` holds 256 doubles.
__device__ void sum_partials(int blk, int nblk, const float2* __restrict__ gacc, int nb, int nn,
                             float2* __restrict__ gsum, const double* __restrict__ loss_part,
                             const double* __restrict__ gs_part, int k, double* __restrict__ loss,
                             float* __restrict__ g_shift, int accumulate, double* red) {
  for (int i = blk * 256 + (int)threadIdx.x; gacc && i < nn; i += nblk * 256) {
    float sx = 0.f, sy = 0.f;
    int bb = 0;
    for (; bb + 8 <= nb; bb += 8) {           // eight loads in flight, added in order
      float2 t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = gacc[(size_t)(bb + u) * nn + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) { sx += t[u].x; sy += t[u].y; }
    }
    for (; bb < nb; ++bb) {
      const float2 t = gacc[(size_t)bb * nn + i];
      sx += t.x;
      sy += t.y;
    }
    gsum[i] = make_float2(sx, sy);
  }
  if (blk != 0) return;
  if (loss) {
    double s = 0.0;
    for (int t = threadIdx.x; t < nb * k; t += 256) s += loss_part[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
  }
  if (g_shift) {
    for (int bb = threadIdx.x; bb < nb; bb += 256) {
      double sy = 0.0, sx = 0.0;
      for (int p = 0; p < k; ++p) {
        sy += gs_part[2 * (bb * k + p)];
        sx += gs_part[2 * (bb * k + p) + 1];
      }
      if (accumulate) { g_shift[2 * bb] += (float)sy; g_shift[2 * bb + 1] += (float)sx; }
      else { g_shift[2 * bb] = (float)sy; g_shift[2 * bb + 1] = (float)sx; }
    }
  }
}

// The arguments of sum_partials for a launch that runs it next to other work.
struct PartialsJob {
  const float2* gacc;
  int nb, nn;
  float2* gsum;
  const double* loss_part;
  const double* gs_part;
  int k;
  double* loss;
  float* g_shift;
  int accumulate;
};

static __global__ void __launch_bounds__(256) reduce_partials_kernel(PartialsJob pj) {
  __shared__ double red[256];
  sum_partials(blockIdx.x, gridDim.x, pj.gacc, pj.nb, pj.nn, pj.gsum, pj.loss_part, pj.gs_part, pj.k, pj.loss,
               pj.g_shift, pj.accumulate, red);
}

// Probe gradient g_p = IDFT(sum_b G_b conj(e_b)) / N^2 from the natural-order
// sum.  One group of K workgroups, as probe_spectrum_kernel.
template <class C>
__global__ void __launch_bounds__(C::THREADS) probe_grad_kernel(const float2* __restrict__ gsum,
                                                                float2* __restrict__ g_probe, int accumulate,
                                                                float2* xbuf, int* counter, int* xcc, int* err) {
  if (probe_idle<C>()) return;
  __shared__ MsShared<C> sh;
  const int part = probe_part<C>();
  Work<C> wk(threadIdx.x, 0, part);
  wk.x.buf = xbuf; wk.x.counter = counter; wk.x.err = err; wk.x.phase = 0; wk.x.local = false;
  const Lane<C>& ln = wk.ln;
  constexpr int N = C::N, NN = N * N;
  build_twiddles<C>(sh.tb, ln.tid);
  __syncthreads();
  if constexpr (C::K > 1) exchange_init<C::K>(wk.x, xcc, part);
  float2 v[C::R];
#pragma unroll
  for (int m = 0; m < C::R; ++m) v[m] = gsum[ln.pos_spec(m) * N + ln.line];
  ifft_line<C, +1>(v, sh.tb, ln);
  xfer<C>(v, sh, wk, false, true);
  ifft_line<C, +1>(v, sh.tb, ln);
  const float s = 1.0f / float(NN);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const int idx = ln.line * N + ln.pos_nat(m);
    float2 g = cscale(v[m], s);
    if (accumulate) g = cadd(g, g_probe[idx]);
    g_probe[idx] = g;
  }
}


// Object gradient from the staged per-position contributions (and, in an
// extra slab of the grid, the per-position partials).  One workgroup per
// kRedTx x kRedTy voxel tile of one slice: it lists, in index
// order, the positions whose chunk overlaps the tile (chunks outside the
// object are skipped, as in the multislice kernel); every voxel then sums the
// contributions of those positions in that order in FP64 and is written once,
// rounded to float32.  A lane covers kRedTx / 64 columns 64 apart and a wave
// kRedTy / 4 rows, so every load instruction reads 64 consecutive floats of
// a staged row; wide tiles split a chunk's 512-byte rows at fewer places
// (each split re-reads one cache line).  Loads of kRedUnroll positions are
// issued together; voxels a chunk does not cover read 0 through the buffer
// range check (an added +0.0 leaves an FP64 sum unchanged).
#ifndef ADORYM_RED_TX
#define ADORYM_RED_TX 256
#endif
#ifndef ADORYM_RED_TY
#define ADORYM_RED_TY 4
#endif
#ifndef ADORYM_RED_UNROLL
#define ADORYM_RED_UNROLL 4
#endif
constexpr int kRedTx = ADORYM_RED_TX, kRedTy = ADORYM_RED_TY, kRedList = 2048, kRedUnroll = ADORYM_RED_UNROLL;
constexpr uint32_t kRedOutside = 0xFFFFFFF0u;   // beyond any plane: reads 0
static __global__ void __launch_bounds__(256) grad_reduce_kernel(const float* __restrict__ stage,
                                                                 const int32_t* __restrict__ corner, int n, int B,
                                                                 int S, int Ly, int Lx, float* __restrict__ g_a,
                                                                 float* __restrict__ g_b, int accumulate,
                                                                 PartialsJob pj) {
  __shared__ int lb[kRedList], lcy[kRedList], lcx[kRedList];
  __shared__ int wave_cnt[4];
  if ((int)blockIdx.z == S) {
    // the last slab of the grid sums the per-position partials meanwhile
    __shared__ double red[256];
    sum_partials(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, pj.gacc, pj.nb, pj.nn, pj.gsum,
                 pj.loss_part, pj.gs_part, pj.k, pj.loss, pj.g_shift, pj.accumulate, red);
    return;
  }
  constexpr int RY = kRedTy / 4;                  // rows per thread
  constexpr int RX = kRedTx / 64;                 // columns per thread
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tx0 = blockIdx.x * kRedTx, ty0 = blockIdx.y * kRedTy, j = blockIdx.z;
  const uint32_t plane_bytes = (uint32_t)(n * n * 4);
  double acc_a[RY][RX], acc_b[RY][RX];
#pragma unroll
  for (int r = 0; r < RY; ++r)
#pragma unroll
    for (int c = 0; c < RX; ++c) acc_a[r][c] = acc_b[r][c] = 0.0;
  for (int w0 = 0; w0 < B; w0 += kRedList) {
    const int w1 = min(B, w0 + kRedList);
    int count = 0;                                  // uniform over the workgroup
    for (int p0 = w0; p0 < w1; p0 += 256) {
      const int p = p0 + threadIdx.x;
      bool hit = false;
      int cy = 0, cx = 0;
      if (p < w1) {
        cy = corner[2 * p];
        cx = corner[2 * p + 1];
        const bool inside = cy >= 0 && cx >= 0 && cy + n <= Ly && cx + n <= Lx;
        hit = inside && cy < ty0 + kRedTy && cy + n > ty0 && cx < tx0 + kRedTx && cx + n > tx0;
      }
      const unsigned long long mask = __ballot(hit);
      if (lane == 0) wave_cnt[wave] = __popcll(mask);
      __syncthreads();
      int at = count + __popcll(mask & ((1ull << lane) - 1ull));
      for (int w = 0; w < wave; ++w) at += wave_cnt[w];
      if (hit) { lb[at] = p; lcy[at] = cy; lcx[at] = cx; }
      count += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
      __syncthreads();
    }
    for (int i0 = 0; i0 < count; i0 += kRedUnroll) {
      float va[kRedUnroll][RY][RX], vb[kRedUnroll][RY][RX];
#pragma unroll
      for (int u = 0; u < kRedUnroll; ++u) {
        const int i = min(i0 + u, count - 1);
        const bool live = i0 + u < count;
        const int pb = __builtin_amdgcn_readfirstlane(lb[i]);
        const int cy = __builtin_amdgcn_readfirstlane(lcy[i]);
        const int cx = __builtin_amdgcn_readfirstlane(lcx[i]);
        const float* base = stage + ((size_t)pb * S + j) * 2 * (size_t)n * n;
        const rsrc_t ra = make_rsrc(base, plane_bytes);
        const rsrc_t rb = make_rsrc(base + (size_t)n * n, plane_bytes);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          const int ly = ty0 + wave + 4 * r - cy;
#pragma unroll
          for (int c = 0; c < RX; ++c) {
            const int lx = tx0 + lane + 64 * c - cx;
            const bool in = live && lx >= 0 && lx < n && ly >= 0 && ly < n;
            const uint32_t off = in ? (uint32_t)(ly * n + lx) * 4 : kRedOutside;
            va[u][r][c] = bload(ra, off, 0);
            vb[u][r][c] = bload(rb, off, 0);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kRedUnroll; ++u)
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
          for (int c = 0; c < RX; ++c) {
            acc_a[r][c] += (double)va[u][r][c];
            acc_b[r][c] += (double)vb[u][r][c];
          }
    }
    __syncthreads();                                // the list is rebuilt for the next window
  }
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = ty0 + wave + 4 * r;
    if (y >= Ly) continue;
#pragma unroll
    for (int c = 0; c < RX; ++c) {
      const int x = tx0 + lane + 64 * c;
      if (x >= Lx) continue;
      const size_t idx = ((size_t)j * Ly + y) * Lx + x;
      double va = acc_a[r][c], vb = acc_b[r][c];
      if (accumulate) { va += (double)g_a[idx]; vb += (double)g_b[idx]; }
      g_a[idx] = (float)va;
      g_b[idx] = (float)vb;
    }
  }
}

// ----------------------------------------------------------------------------
// Host side
// ----------------------------------------------------------------------------
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int kMaxSplit = 8;   // largest K any kernel uses

struct WsLayout {
  size_t q, gsum, loss_part, gs_part, counters, xcc, aux, gacc, ckpt, recomp, xbuf, stage, total;
  int nslots, nrec;
};

// Workspace of a loss+gradient call; forward_only: of a forward call (no
// checkpoints, partials or staging).
inline WsLayout ws_layout(const adorym_geom* g, int batch, bool forward_only = false) {
  WsLayout w{};
  const size_t nn = (size_t)g->n * g->n;
  const int S = g->n_slices, C = g->ckpt_every;
  w.nslots = (S - 1) / C + 1 + (((S - 1) % C) != 0 ? 1 : 0);
  w.nrec = std::max(0, std::min(C - 1, S - 2));      // interior slices of a segment
  size_t off = 0;
  w.q = off; off += align256(nn * sizeof(float2));
  w.gsum = off; off += align256(nn * sizeof(float2));
  w.loss_part = off; off += align256((size_t)batch * kMaxSplit * sizeof(double));
  w.gs_part = off; off += align256((size_t)batch * kMaxSplit * 2 * sizeof(double));
  w.counters = off; off += align256((size_t)(batch + S) * sizeof(int));   // then the S slice bounds
  w.xcc = off; off += align256((size_t)batch * kMaxSplit * sizeof(int));
  w.aux = off; off += align256(64 * sizeof(int));   // probe kernels: 2 counters + XCD ids
  w.xbuf = off; off += align256((size_t)batch * 4 * nn * sizeof(float2));
  w.gacc = off; if (!forward_only) off += align256((size_t)batch * nn * sizeof(float2));
  w.ckpt = off; if (!forward_only) off += align256((size_t)batch * w.nslots * nn * sizeof(float2));
  w.recomp = off; if (!forward_only) off += align256((size_t)batch * w.nrec * nn * sizeof(float2));
  w.stage = off; if (!forward_only) off += align256((size_t)batch * S * 2 * nn * sizeof(float));
  w.total = off;
  return w;
}

inline adorym_status set_err(adorym_ctx* ctx, adorym_status st, const char* what) {
  if (ctx) snprintf(ctx->msg, sizeof(ctx->msg), "%s", what);
  return st;
}

inline adorym_status check_geom(adorym_ctx* ctx, const adorym_geom* g, int batch) {
  if (!ctx) return ADORYM_EINVAL;
  if (!g) return set_err(ctx, ADORYM_EINVAL, "geometry is NULL");
  if (!adorym_supports_n(g->n)) return set_err(ctx, ADORYM_EUNSUPPORTED, "probe size N has no kernel");
  if (g->n_slices < 1) return set_err(ctx, ADORYM_EINVAL, "n_slices must be >= 1");
  if (g->obj_ny < g->n || g->obj_nx < g->n) return set_err(ctx, ADORYM_EINVAL, "object smaller than the probe");
  if ((size_t)g->obj_ny * g->obj_nx * 4 > 0xFFFFFFF0ull)
    return set_err(ctx, ADORYM_EUNSUPPORTED, "one object slice exceeds 4 GiB");
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


template <class C, bool LOSS, bool VAR = false, bool NF = false, bool SPLIT = false>
void launch_ms(const MsParams& P, int repr, hipStream_t st) {
  // XCD-aware grid: ceil(B/8) groups per XCD, K slots per group
  const dim3 grid(((P.B + 7) / 8) * 8 * C::K), block(C::THREADS);
  if (repr == ADORYM_OBJ_DELTA_BETA)
    hipLaunchKernelGGL((multislice_kernel<C, ADORYM_OBJ_DELTA_BETA, LOSS, VAR, NF, SPLIT>), grid, block, 0, st, P);
  else
    hipLaunchKernelGGL((multislice_kernel<C, ADORYM_OBJ_REAL_IMAG, LOSS, VAR, NF, SPLIT>), grid, block, 0, st, P);
}

// Kernel parameters of one job; `ws` is its workspace (adorym_workspace_size).
template <int N, int L>
MsParams make_params(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, int batch,
                     const int32_t* corner, const float* shift, const float* i_meas, void* ws, bool with_probe_grad,
                     float* g_a, float* g_b, float* intensity) {
  const WsLayout w = ws_layout(g, batch);
  char* base = static_cast<char*>(ws);
  MsParams P{};
  P.a = a; P.b = b;
  P.q = reinterpret_cast<const float2*>(base + w.q);
  P.corner = corner; P.shift = shift; P.i_meas = i_meas; P.intensity = intensity;
  P.i_total = ctx->i_total;
  P.g_a = g_a; P.g_b = g_b;
  P.gstage = g_a ? reinterpret_cast<float*>(base + w.stage) : nullptr;
  P.ckpt = reinterpret_cast<float2*>(base + w.ckpt);
  P.recomp = reinterpret_cast<float2*>(base + w.recomp);
  P.gacc = with_probe_grad ? reinterpret_cast<float2*>(base + w.gacc) : nullptr;
  P.loss_part = reinterpret_cast<double*>(base + w.loss_part);
  P.gs_part = reinterpret_cast<double*>(base + w.gs_part);
  P.xbuf = reinterpret_cast<float2*>(base + w.xbuf);
  P.counters = reinterpret_cast<int*>(base + w.counters);
  P.absorb = reinterpret_cast<const float*>(base + w.counters) + batch;
  P.xcc = reinterpret_cast<int*>(base + w.xcc);
  P.err = ctx->d_err;
  P.B = batch; P.S = g->n_slices; P.Ly = g->obj_ny; P.Lx = g->obj_nx;
  P.ckpt_every = g->ckpt_every; P.nslots = w.nslots; P.nrec = w.nrec;
  P.loss = g->loss;
  P.kdz = (float)(2.0 * M_PI / g->wavelength_m * g->slice_dz_m);
  P.chirp = g->wavelength_m * g->slice_dz_m / (g->pixel_m * g->pixel_m);
  P.eps = g->eps;
  P.adj_scale = 1.0f;
  P.inv_n = 1.0 / ((double)batch * g->n * g->n);
  return P;
}

// Tile of the one-group probe kernels: the whole field in one workgroup for
// small probes, else split over four workgroups (four CUs of one XCD; for
// N = 128 that is faster than one 1024-thread workgroup with LDS transposes).
template <int N, int L>
using ProbeCfg = TileCfg<N, L, (N >= 128 ? 4 : 1)>;

// Per-job work before the multislice kernel: clear the barrier counters,
// then one launch for the probe spectrum and, before a reverse sweep that
// steps backwards through slices (`reverse`), the per-slice absorption
// bounds.
template <int N, int L>
void launch_prologue(const MsParams& P, const float* probe, const adorym_geom* g, hipStream_t st, bool reverse) {
  using PC = ProbeCfg<N, L>;
  const WsLayout w = ws_layout(g, P.B);
  int* aux = reinterpret_cast<int*>(reinterpret_cast<char*>(P.counters) - w.counters + w.aux);
  // the multislice counters and slice bounds, the XCD ids and the probe
  // kernels' counters lie in one run of the workspace
  hipLaunchKernelGGL(reset_ints_kernel, dim3(1), dim3(256), 0, st, P.counters,
                     (int)((w.aux - w.counters) / sizeof(int)) + 64);
  AbsorbJob ab{};
  unsigned blocks = probe_grid<PC>();
  if (reverse && P.ckpt_every > 1 && P.S > 2) {
    ab.a = P.a;
    ab.b = P.b;
    ab.plane = (size_t)P.Ly * P.Lx;
    ab.kdz = P.kdz;
    ab.out = reinterpret_cast<unsigned*>(P.counters + P.B);
    ab.parts = (int)std::min<size_t>(64, (ab.plane + 64 * PC::THREADS - 1) / (64 * PC::THREADS));
    ab.repr = g->obj_repr;
    blocks += (unsigned)(ab.parts * P.S);
  }
  hipLaunchKernelGGL((probe_spectrum_kernel<PC>), dim3(blocks), dim3(PC::THREADS), 0, st,
                     reinterpret_cast<const float2*>(probe), const_cast<float2*>(P.q), P.xbuf, aux, aux + 8,
                     P.err, ab);
}

// Per-job work after it: loss, shift gradients, probe gradient; with object
// gradients the partial sums run in the object-gradient reduction's launch.
template <int N, int L>
void launch_epilogue(const MsParams& P, void* ws, const adorym_geom* g, double* loss, float* g_probe,
                     float* g_shift, hipStream_t st, const Defocus* df = nullptr) {
  using PC = ProbeCfg<N, L>;
  const WsLayout w = ws_layout(g, P.B);
  int* aux = reinterpret_cast<int*>(static_cast<char*>(ws) + w.aux);
  float2* gsum = reinterpret_cast<float2*>(static_cast<char*>(ws) + w.gsum);
  const int accumulate = (g->flags & ADORYM_ACCUMULATE_GRADS) ? 1 : 0;
  const int nn = N * N;
  const PartialsJob pj{P.gacc, P.B, nn, gsum, P.loss_part, P.gs_part, P.ksplit, loss, g_shift, accumulate};
  if (P.gstage) {
    const dim3 grid((P.Lx + kRedTx - 1) / kRedTx, (P.Ly + kRedTy - 1) / kRedTy, P.S + 1);
    hipLaunchKernelGGL(grad_reduce_kernel, grid, dim3(256), 0, st, P.gstage, P.corner, N, P.B, P.S, P.Ly, P.Lx,
                       P.g_a, P.g_b, accumulate, pj);
  } else {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((nn + 255) / 256), dim3(256), 0, st, pj);
  }
  if (df && P.gacc) {
    // the per-position probe partials are consumed by now: their first bytes
    // hold the defocus-gradient shares
    double* part = reinterpret_cast<double*>(P.gacc);
    hipLaunchKernelGGL(defocus_grad_kernel, dim3(kDefocusParts), dim3(256), 0, st, gsum, P.q, N, df->c0, df->dist,
                       part);
    hipLaunchKernelGGL(defocus_finish_kernel, dim3(1), dim3(kDefocusParts), 0, st, part, df->g_dist, accumulate);
  }
  if (g_probe)
    hipLaunchKernelGGL((probe_grad_kernel<PC>), dim3(probe_grid<PC>()), dim3(PC::THREADS), 0, st, gsum,
                       reinterpret_cast<float2*>(g_probe), accumulate, P.xbuf, aux + 1, aux + 16, P.err);
}

// Lanes per line of the one-group probe kernels and the job parameters: one
// value per probe size, whatever tile the multislice kernel of a call uses,
// so that every path computes the probe spectrum and gradient identically.
template <int N>
constexpr int probe_lanes() { return N == 64 ? 4 : 8; }

// Deterministic mode runs with one fixed split per probe size, so that a
// job's results do not depend on the split chosen for other calls.
constexpr int det_split(int n) { return n == 192 ? 6 : (n == 128 ? 4 : 1); }

// One probe size N with lanes-per-line L and split K.
template <int N, int L, int K>
adorym_status run(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                  const int32_t* corner, const float* shift, int batch, const float* i_meas, void* ws,
                  double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift, float* intensity,
                  bool with_loss, const Defocus* df = nullptr) {
  using C = TileCfg<N, L, K>;
  const bool probe_partials = g_probe != nullptr || (df && df->g_dist);
  MsParams P = make_params<N, probe_lanes<N>()>(ctx, g, a, b, batch, corner, shift, i_meas, ws, probe_partials,
                                    with_loss ? g_a : nullptr, with_loss ? g_b : nullptr, intensity);
  P.ksplit = K;
  hipStream_t st = ctx->stream;
  const bool timed = ctx->prof && ctx->ev_used + 2 <= (int)ctx->ev.size();
  launch_prologue<N, probe_lanes<N>()>(P, probe, g, st, with_loss);
  if (df)
    hipLaunchKernelGGL(defocus_spectrum_kernel, dim3((N * N + 255) / 256), dim3(256), 0, st,
                       const_cast<float2*>(P.q), N, df->c0, df->dist);
  if (timed) (void)hipEventRecord(ctx->ev[ctx->ev_used], st);
  if (with_loss) launch_ms<C, true>(P, g->obj_repr, st);
  else launch_ms<C, false>(P, g->obj_repr, st);
  if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
  if (with_loss) launch_epilogue<N, probe_lanes<N>()>(P, ws, g, loss, g_probe, g_shift, st, df);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return ADORYM_OK;
}

// Gap gradients dL/dd_j = scale * sum of the (position, part) partials of
// gap j, one workgroup per gap: a fixed strided split over the threads and a
// fixed-order tree, in FP64 (bitwise reproducible).
static __global__ void __launch_bounds__(256) gap_reduce_kernel(const double* __restrict__ part, int nbk, int ngaps,
                                                                double scale, double* __restrict__ g_gaps,
                                                                int accumulate) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nbk; i += blockDim.x) s += part[(size_t)i * ngaps + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) g_gaps[j] = accumulate ? g_gaps[j] + scale * red[0] : scale * red[0];
}

// Workspace of the unequal-spacing calls: that of the uniform call plus the
// gap-gradient partials.
inline size_t gaps_ws_size(const adorym_geom* g, int batch, bool forward_only) {
  const size_t base = ws_layout(g, batch, forward_only).total;
  if (forward_only) return base;
  return base + align256((size_t)batch * kMaxSplit * std::max(g->n_slices - 1, 1) * sizeof(double));
}

// Unequal slice spacing (sparse multislice): as run, with the Fresnel table
// rebuilt for every gap and, with the loss, the gap gradients.
template <int N, int L, int K>
adorym_status run_gaps(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                       const int32_t* corner, const float* shift, int batch, const double* gaps, const float* i_meas,
                       void* ws, double* loss, float* g_a, float* g_b, float* g_probe, float* g_shift,
                       double* g_gaps, float* intensity, bool with_loss) {
  using C = TileCfg<N, L, K>;
  MsParams P = make_params<N, probe_lanes<N>()>(ctx, g, a, b, batch, corner, shift, i_meas, ws, g_probe != nullptr,
                                    with_loss ? g_a : nullptr, with_loss ? g_b : nullptr, intensity);
  P.ksplit = K;
  P.gaps = gaps;
  P.chirp_per_m = g->wavelength_m / (g->pixel_m * g->pixel_m);
  P.gd_part = with_loss ? reinterpret_cast<double*>(static_cast<char*>(ws) + ws_layout(g, batch).total) : nullptr;
  hipStream_t st = ctx->stream;
  const bool timed = ctx->prof && ctx->ev_used + 2 <= (int)ctx->ev.size();
  launch_prologue<N, probe_lanes<N>()>(P, probe, g, st, with_loss);
  if (timed) (void)hipEventRecord(ctx->ev[ctx->ev_used], st);
  if (with_loss) launch_ms<C, true, true>(P, g->obj_repr, st);
  else launch_ms<C, false, true>(P, g->obj_repr, st);
  if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
  if (with_loss) {
    launch_epilogue<N, probe_lanes<N>()>(P, ws, g, loss, g_probe, g_shift, st);
    if (g_gaps && P.S > 1) {
      const double scale = -M_PI * P.chirp_per_m / ((double)N * N * N);
      hipLaunchKernelGGL(gap_reduce_kernel, dim3(P.S - 1), dim3(256), 0, st, P.gd_part, P.B * K, P.S - 1, scale,
                         g_gaps, (g->flags & ADORYM_ACCUMULATE_GRADS) ? 1 : 0);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return ADORYM_OK;
}

// ---- Near field (Fresnel propagation to the detector) ----------------------
// Transfer functions to the detector and d(phase)/d(distance), in FP64:
// paraxial H1 = exp(i pi lambda d |nu|^2); Sommerfeld H2 without its global
// phase exp(-i k d) (it does not change an intensity), i.e.
// exp(i k d x / (sqrt(1 - x) + 1)), x = lambda^2 |nu|^2 < 1, and 0 for the
// evanescent x >= 1.  The phase is reduced modulo 2 pi in FP64.
static __global__ void nf_table_kernel(int n, double lambda, double dx, int kind, const double* __restrict__ dist,
                                       int n_dist, float2* __restrict__ h, float* __restrict__ dph) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int ka = i / n, kb = i % n;
  const double fa = double(ka < (n + 1) / 2 ? ka : ka - n) / (n * dx);
  const double fb = double(kb < (n + 1) / 2 ? kb : kb - n) / (n * dx);
  const double nu2 = fa * fa + fb * fb;
  double g = 0.0;                 // phase per metre of distance
  bool pass = true;
  if (kind == ADORYM_PROP_PARAXIAL) {
    g = M_PI * lambda * nu2;
  } else {
    const double x = lambda * lambda * nu2;
    if (x >= 1.0) pass = false;
    else g = (2.0 * M_PI / lambda) * x / (sqrt(1.0 - x) + 1.0);
  }
  dph[i] = (float)g;
  for (int d = 0; d < n_dist; ++d) {
    double sn, cs;
    sincos(fmod(g * dist[d], 2.0 * M_PI), &sn, &cs);
    h[(size_t)d * n * n + i] = pass ? make_float2((float)cs, (float)sn) : make_float2(0.f, 0.f);
  }
}

// dL/d(distance d) = sum of the partials of the positions with index d, in
// position order (one workgroup per distance).
static __global__ void __launch_bounds__(256) dist_reduce_kernel(const double* __restrict__ part,
                                                                 const int32_t* __restrict__ idx, int nb, int k,
                                                                 double* __restrict__ g_dist, int accumulate) {
  __shared__ double red[256];
  const int d = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256)
    if (idx[b] == d)
      for (int p = 0; p < k; ++p) s += part[b * k + p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) g_dist[d] = accumulate ? g_dist[d] + red[0] : red[0];
}

// Workspace of the near-field calls: that of the far-field call, then the
// distance partials, the detector spectra, the transfer functions and the
// phase derivative.
struct NfLayout { size_t part, spec, h, dph, total; };
inline NfLayout nf_layout(const adorym_geom* g, int batch, int n_dist) {
  NfLayout l{};
  const size_t nn = (size_t)g->n * g->n;
  size_t off = ws_layout(g, batch).total;
  l.part = off; off += align256((size_t)batch * kMaxSplit * sizeof(double));
  l.spec = off; off += align256((size_t)batch * nn * sizeof(float2));
  l.h = off; off += align256((size_t)n_dist * nn * sizeof(float2));
  l.dph = off; off += align256(nn * sizeof(float));
  l.total = off;
  return l;
}

template <int N, int L, int K>
adorym_status run_nf(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                     const int32_t* corner, const float* shift, int batch, int kind, const double* dist, int n_dist,
                     const int32_t* dist_idx, const float* i_meas, void* ws, double* loss, float* g_a, float* g_b,
                     float* g_probe, float* g_shift, double* g_dist, float* intensity, bool with_loss) {
  using C = TileCfg<N, L, K>;
  MsParams P = make_params<N, probe_lanes<N>()>(ctx, g, a, b, batch, corner, shift, i_meas, ws, g_probe != nullptr,
                                    with_loss ? g_a : nullptr, with_loss ? g_b : nullptr, intensity);
  P.ksplit = K;
  const NfLayout l = nf_layout(g, batch, n_dist);
  char* base = static_cast<char*>(ws);
  P.nd_part = reinterpret_cast<double*>(base + l.part);
  P.nf_spec = reinterpret_cast<float2*>(base + l.spec);
  P.nf_h = reinterpret_cast<const float2*>(base + l.h);
  P.nf_dph = reinterpret_cast<const float*>(base + l.dph);
  P.nf_idx = dist_idx;
  P.n_dist = n_dist;
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(nf_table_kernel, dim3((N * N + 255) / 256), dim3(256), 0, st, N, g->wavelength_m, g->pixel_m,
                     kind, dist, n_dist, reinterpret_cast<float2*>(base + l.h), reinterpret_cast<float*>(base + l.dph));
  const bool timed = ctx->prof && ctx->ev_used + 2 <= (int)ctx->ev.size();
  launch_prologue<N, probe_lanes<N>()>(P, probe, g, st, with_loss);
  if (timed) (void)hipEventRecord(ctx->ev[ctx->ev_used], st);
  if (with_loss) launch_ms<C, true, false, true>(P, g->obj_repr, st);
  else launch_ms<C, false, false, true>(P, g->obj_repr, st);
  if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
  if (with_loss) {
    launch_epilogue<N, probe_lanes<N>()>(P, ws, g, loss, g_probe, g_shift, st);
    if (g_dist)
      hipLaunchKernelGGL(dist_reduce_kernel, dim3(n_dist), dim3(256), 0, st, P.nd_part, dist_idx, P.B, K, g_dist,
                         (g->flags & ADORYM_ACCUMULATE_GRADS) ? 1 : 0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return ADORYM_OK;
}

// Loss of predicted intensities (per-pixel terms in FP32 as in the fused
// kernel, the mean over the n pixels in FP64): a fixed grid-stride split and
// a fixed-order tree per workgroup, partials summed by finish_loss_kernel.
constexpr int kLossBlocks = 256;
static __global__ void __launch_bounds__(256) loss_value_kernel(const float* __restrict__ ip,
                                                                const float* __restrict__ im, size_t n, int kind,
                                                                float eps, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float p = ip[i], m = im[i];
    float term;
    if (kind == ADORYM_LOSS_GAUSSIAN) {
      const float d = sqrtf(p + eps) - sqrtf(m + eps);
      term = d * d;
    } else {
      term = p - m * logf(p + eps);
    }
    s += (double)term;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
static __global__ void __launch_bounds__(256) finish_loss_kernel(const double* __restrict__ part, double inv_n,
                                                                 double* __restrict__ loss) {
  __shared__ double red[256];
  red[threadIdx.x] = part[threadIdx.x];      // kLossBlocks == 256
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv_n;
}

// ---- Split evaluation (several probe modes) ------------------------------
// Per-mode storage between the passes: the checkpoints and the exit wave.
inline size_t split_ckpt_bytes(const adorym_geom* g, int batch) {
  const WsLayout w = ws_layout(g, batch);
  return align256((size_t)batch * w.nslots * g->n * g->n * sizeof(float2));
}
inline size_t split_exit_bytes(const adorym_geom* g, int batch) {
  return align256((size_t)batch * g->n * g->n * sizeof(float2));
}

// One pass of a split evaluation: the forward pass (with_loss false: stores
// checkpoints and the exit wave, writes the intensity) or the loss pass
// (resumes from them).  `ws` is a loss-and-gradient workspace.
template <int N, int L, int K>
adorym_status run_split(adorym_ctx* ctx, const adorym_geom* g, const float* a, const float* b, const float* probe,
                        const int32_t* corner, const float* shift, int batch, const float* i_meas, void* ws,
                        float2* ckpt, float2* exit_wave, double* loss, float* g_a, float* g_b, float* g_probe,
                        float* g_shift, float* intensity, bool with_loss, float adj_scale) {
  using C = TileCfg<N, L, K>;
  MsParams P = make_params<N, probe_lanes<N>()>(ctx, g, a, b, batch, corner, shift, i_meas, ws, g_probe != nullptr,
                                    with_loss ? g_a : nullptr, with_loss ? g_b : nullptr, intensity);
  P.ksplit = K;
  P.ckpt = ckpt;
  P.exit_wave = exit_wave;
  P.adj_scale = adj_scale;
  hipStream_t st = ctx->stream;
  const bool timed = ctx->prof && ctx->ev_used + 2 <= (int)ctx->ev.size();
  launch_prologue<N, probe_lanes<N>()>(P, probe, g, st, with_loss);
  if (timed) (void)hipEventRecord(ctx->ev[ctx->ev_used], st);
  if (with_loss) launch_ms<C, true, false, false, true>(P, g->obj_repr, st);
  else launch_ms<C, false, false, false, true>(P, g->obj_repr, st);
  if (timed) { (void)hipEventRecord(ctx->ev[ctx->ev_used + 1], st); ctx->ev_used += 2; }
  if (with_loss) launch_epilogue<N, probe_lanes<N>()>(P, ws, g, loss, g_probe, g_shift, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, ADORYM_EDEVICE, hipGetErrorString(e));
  return ADORYM_OK;
}

// The persistent multi-job kernel of one probe-size class (device tables
// prepared by the plan).
template <int N, int L, int K>
void launch_batched(const MsParams* jobs, const int2* items, int n_items, int* ticket, int* mailbox, int* counters,
                    int* xcc, float2* xbuf, int* err, int groups, int repr, hipStream_t st) {
  using C = TileCfg<N, L, K>;
  const dim3 grid(groups * K), block(C::THREADS);
  if (repr == ADORYM_OBJ_DELTA_BETA)
    hipLaunchKernelGGL((multislice_batched_kernel<C, ADORYM_OBJ_DELTA_BETA>), grid, block, 0, st, jobs, items,
                       n_items, ticket, mailbox, counters, xcc, xbuf, err);
  else
    hipLaunchKernelGGL((multislice_batched_kernel<C, ADORYM_OBJ_REAL_IMAG>), grid, block, 0, st, jobs, items,
                       n_items, ticket, mailbox, counters, xcc, xbuf, err);
}

}  // namespace adorym_ms

// Explicit instantiation helpers
#define ADORYM_BATCHED_SIGNATURE(N_, L_, K_) \
  void adorym_ms::launch_batched<N_, L_, K_>(const adorym_ms::MsParams*, const int2*, int, int*, int*, int*, int*, \
                                              float2*, int*, int, int, hipStream_t)
#define ADORYM_PROLOGUE_SIGNATURE(N_, L_) \
  void adorym_ms::launch_prologue<N_, L_>(const adorym_ms::MsParams&, const float*, const adorym_geom*, hipStream_t, \
                                          bool)
#define ADORYM_EPILOGUE_SIGNATURE(N_, L_) \
  void adorym_ms::launch_epilogue<N_, L_>(const adorym_ms::MsParams&, void*, const adorym_geom*, double*, float*, \
                                          float*, hipStream_t, const adorym_ms::Defocus*)
#define ADORYM_PARAMS_SIGNATURE(N_, L_) \
  adorym_ms::MsParams adorym_ms::make_params<N_, L_>(adorym_ctx*, const adorym_geom*, const float*, \
                                                        const float*, int, const int32_t*, const float*, \
                                                        const float*, void*, bool, float*, float*, float*)
#define ADORYM_RUN_SPLIT_SIGNATURE(N_, L_, K_) \
  adorym_status adorym_ms::run_split<N_, L_, K_>(adorym_ctx*, const adorym_geom*, const float*, const float*, \
                                                 const float*, const int32_t*, const float*, int, const float*, \
                                                 void*, float2*, float2*, double*, float*, float*, float*, float*, \
                                                 float*, bool, float)
#define ADORYM_RUN_NF_SIGNATURE(N_, L_, K_) \
  adorym_status adorym_ms::run_nf<N_, L_, K_>(adorym_ctx*, const adorym_geom*, const float*, const float*, \
                                              const float*, const int32_t*, const float*, int, int, const double*, \
                                              int, const int32_t*, const float*, void*, double*, float*, float*, \
                                              float*, float*, double*, float*, bool)
#define ADORYM_RUN_GAPS_SIGNATURE(N_, L_, K_) \
  adorym_status adorym_ms::run_gaps<N_, L_, K_>(adorym_ctx*, const adorym_geom*, const float*, const float*, \
                                                const float*, const int32_t*, const float*, int, const double*, \
                                                const float*, void*, double*, float*, float*, float*, float*, \
                                                double*, float*, bool)
#define ADORYM_RUN_SIGNATURE(N_, L_, K_) \
  adorym_status adorym_ms::run<N_, L_, K_>(adorym_ctx*, const adorym_geom*, const float*, const float*, const float*, \
                                           const int32_t*, const float*, int, const float*, void*, double*, float*, \
                                           float*, float*, float*, float*, bool, const adorym_ms::Defocus*)
