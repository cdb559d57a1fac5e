// tile.hpp -- register/LDS tile engine for N x N complex wavefields on gfx950.
//
// One workgroup owns one N x N complex64 field (a probe position's
// wavefield).  The field lives in VGPRs: each thread holds R complex values
// of one "line" (a row or a column of the field), and the L lanes of a lane
// group hold one whole line (N = L * R).  A wave holds 64/L lines.
//
//   line layout ROW: the thread's line is row y, its values are columns x
//   line layout COL: the thread's line is column x, its values are rows y
//
// Along a line, lane l (logical index q = Lg(l)) register m holds position
//   natural order : n = q + L*m                       (strided)
//   spectral order: k = R*bitrev_L(q) + m             (after fft_line)
//
// A 1D DFT along the line is an R-point DFT in registers, a twiddle
// W_N^{q*k2}, and an L-point DFT across the lanes of the group (radix 2,
// decimation in frequency, exchanges by DPP).  For L = 8 lanes 4..7 hold
// logical indices 7..4, so the span-4 partner is DPP row_half_mirror and the
// span-2/1 partners are quad permutations: every exchange is one DPP move.
//
// The paraxial Fresnel kernel exp(i pi lambda dz (nu_y^2 + nu_x^2)) is the
// product of two 1D kernels, so the 2D propagation F^-1 H F is a 1D
// propagation along rows times one along columns, and the two commute.
// A slice step therefore needs a single LDS transpose: rows are propagated
// in ROW layout, the field is transposed, columns are propagated in COL
// layout, and the next slice is modulated in COL layout (and so on,
// alternating).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adorym {

// ----------------------------------------------------------------------------
// Complex helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ----------------------------------------------------------------------------
// Compile-time twiddles W_M^e = exp(SIGN * 2 pi i e / M), evaluated in double
// by an octant-reduced Taylor series (no library trigonometry involved).
// ----------------------------------------------------------------------------
constexpr double kPiD = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 16; ++k) { term *= -x2 / double((2 * k) * (2 * k + 1)); sum += term; }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 16; ++k) { term *= -x2 / double((2 * k - 1) * (2 * k)); sum += term; }
  return sum;
}
// cos and sin of 2 pi e / m for integers, exact at multiples of pi/4.
struct CS { double c, s; };
constexpr CS cs_turn(long e, long m) {
  long r = ((e % m) + m) % m;      // [0, m)
  long q = (4 * r) / m;            // quadrant 0..3
  long rem = 4 * r - q * m;        // angle within quadrant = (pi/2) rem / m
  double c = 0, s = 0;
  if (2 * rem <= m) {
    double a = (kPiD / 2.0) * double(rem) / double(m);
    c = taylor_cos(a); s = taylor_sin(a);
  } else {
    double a = (kPiD / 2.0) * double(m - rem) / double(m);
    c = taylor_sin(a); s = taylor_cos(a);
  }
  if (rem == 0) { c = 1.0; s = 0.0; }
  // rotate by q quarter turns
  for (long i = 0; i < q; ++i) { double t = c; c = -s; s = t; }
  return CS{c, s};
}

template <long E, int M, int SIGN>
struct Tw {
  static constexpr long r = ((E % M) + M) % M;
  static constexpr CS cs = cs_turn(r, M);
  static constexpr float re = float(cs.c);
  static constexpr float im = float(SIGN > 0 ? cs.s : -cs.s);
  // classification for cheap special cases
  static constexpr bool one = (r == 0);
  static constexpr bool minus_one = (2 * r == M);
  static constexpr bool quarter = (4 * r == M) || (4 * r == 3 * M);  // +-i
};

// v * W_M^E with the trivial cases handled without multiplies.
template <long E, int M, int SIGN>
__device__ __forceinline__ float2 twmul(float2 v) {
  using T = Tw<E, M, SIGN>;
  if constexpr (T::one) {
    return v;
  } else if constexpr (T::minus_one) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (T::quarter) {
    // multiply by i*T::im (T::im = +-1)
    if constexpr (T::im > 0) return make_float2(-v.y, v.x);
    else return make_float2(v.y, -v.x);
  } else {
    constexpr float c = T::re, s = T::im;
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// ----------------------------------------------------------------------------
// Compile-time loops
// ----------------------------------------------------------------------------
template <int I, int END>
struct CFor {
  template <class F>
  static __device__ __forceinline__ void run(F&& f) {
    if constexpr (I < END) {
      f(std::integral_constant<int, I>{});
      CFor<I + 1, END>::run(f);
    }
  }
};

// ----------------------------------------------------------------------------
// In-register DFT of M points over v[OFF + ST*i], natural order in and out.
// Mixed radix: M = P * Q with P the first factor in {4, 2, 3}:
//   X[Q k1 + k2] = sum_n1 W_P^{n1 k1} W_M^{n1 k2} sum_n2 x[n1 + P n2] W_Q^{n2 k2}
// ----------------------------------------------------------------------------
template <int M> struct FirstFactor {
  static constexpr int value = (M % 4 == 0 && M != 8) ? 4 : (M % 2 == 0 ? 2 : 3);
};

template <int M, int SIGN, int ST, int OFF, int CAP>
struct Dft {
  static __device__ __forceinline__ void run(float2 (&v)[CAP]) {
    if constexpr (M == 1) {
      return;
    } else if constexpr (M == 2) {
      float2 a = v[OFF], b = v[OFF + ST];
      v[OFF] = cadd(a, b);
      v[OFF + ST] = csub(a, b);
    } else if constexpr (M == 3) {
      // W_3 = -1/2 + SIGN i sqrt(3)/2
      constexpr float h = 0.8660254037844386f;  // sqrt(3)/2
      float2 a = v[OFF], b = v[OFF + ST], c = v[OFF + 2 * ST];
      float2 s = cadd(b, c), d = csub(b, c);
      float2 m = make_float2(a.x - 0.5f * s.x, a.y - 0.5f * s.y);
      // i * SIGN * h * d
      float2 r = SIGN > 0 ? make_float2(-h * d.y, h * d.x) : make_float2(h * d.y, -h * d.x);
      v[OFF] = cadd(a, s);
      v[OFF + ST] = cadd(m, r);
      v[OFF + 2 * ST] = csub(m, r);
    } else if constexpr (M == 4) {
      float2 a = v[OFF], b = v[OFF + ST], c = v[OFF + 2 * ST], d = v[OFF + 3 * ST];
      float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = csub(b, d);
      // W_4^1 = SIGN * i
      float2 jd1 = SIGN > 0 ? make_float2(-d1.y, d1.x) : make_float2(d1.y, -d1.x);
      v[OFF] = cadd(s0, s1);
      v[OFF + ST] = cadd(d0, jd1);
      v[OFF + 2 * ST] = csub(s0, s1);
      v[OFF + 3 * ST] = csub(d0, jd1);
    } else {
      constexpr int P = FirstFactor<M>::value;
      constexpr int Q = M / P;
      // Q-point DFTs over n2 for each n1 (elements n1 + P n2)
      CFor<0, P>::run([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        Dft<Q, SIGN, ST * P, OFF + ST * n1, CAP>::run(v);
      });
      // twiddles W_M^{n1 k2} on element n1 + P k2
      CFor<1, P>::run([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        CFor<1, Q>::run([&](auto k2c) {
          constexpr int k2 = decltype(k2c)::value;
          v[OFF + ST * (n1 + P * k2)] = twmul<long(n1) * k2, M, SIGN>(v[OFF + ST * (n1 + P * k2)]);
        });
      });
      // P-point DFTs over n1 for each k2 (elements n1 + P k2, stride 1 in n1)
      CFor<0, Q>::run([&](auto k2c) {
        constexpr int k2 = decltype(k2c)::value;
        Dft<P, SIGN, ST, OFF + ST * P * k2, CAP>::run(v);
      });
      // element k1 + P k2 holds X[Q k1 + k2]: permute to natural order
      float2 t[M];
      CFor<0, P>::run([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        CFor<0, Q>::run([&](auto k2c) {
          constexpr int k2 = decltype(k2c)::value;
          t[Q * k1 + k2] = v[OFF + ST * (k1 + P * k2)];
        });
      });
      CFor<0, M>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        v[OFF + ST * i] = t[i];
      });
    }
  }
};

// ----------------------------------------------------------------------------
// DPP lane exchanges within a lane group of L lanes (L = 4, 8 or 16)
// ----------------------------------------------------------------------------
enum : int {
  kDppQuadXor1 = 0xB1,     // quad_perm [1,0,3,2]
  kDppQuadXor2 = 0x4E,     // quad_perm [2,3,0,1]
  kDppHalfMirror = 0x141,  // row_half_mirror: lane i <- lane 7-i within 8
  kDppMirror = 0x140,      // row_mirror: lane i <- lane 15-i within 16
};

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ float2 dpp2(float2 v) {
  return make_float2(dpp<CTRL>(v.x), dpp<CTRL>(v.y));
}
template <int L, int H>
__device__ __forceinline__ float2 partner(float2 v) {
  if constexpr (L == 16 && H == 8) return dpp2<kDppMirror>(v);
  else if constexpr (L >= 8 && H == 4) return dpp2<kDppHalfMirror>(v);
  else if constexpr (H == 2) return dpp2<kDppQuadXor2>(v);
  else return dpp2<kDppQuadXor1>(v);
}

// Fused cross-lane butterfly half: x <- x + s * partner(x), one
// v_fmac_f32_dpp per value (the partner read through DPP as the
// multiplicand), where a DPP move and a multiply-add would take two
// instructions.  The compiler does not form this instruction itself, so it
// is written out; its operands are plain registers.  A DPP read of a VGPR
// needs two wait states after the VALU instruction that wrote it, which the
// compiler cannot see across inline assembly: dpp_enter orders every value's
// producer before an s_nop 1, dpp_leave puts an s_nop 1 after the last DPP
// write and orders every consumer after it.  Full waves only (every lane
// active), as all tile code.
#ifndef ADORYM_FUSED_DPP
#define ADORYM_FUSED_DPP 1
#endif
template <int L, int H>
__device__ __forceinline__ void dpp_fmac(float& x, float s) {
  if constexpr (L == 16 && H == 8)
    asm volatile("v_fmac_f32_dpp %0, %0, %1 row_mirror row_mask:0xf bank_mask:0xf" : "+v"(x) : "v"(s));
  else if constexpr (L >= 8 && H == 4)
    asm volatile("v_fmac_f32_dpp %0, %0, %1 row_half_mirror row_mask:0xf bank_mask:0xf" : "+v"(x) : "v"(s));
  else if constexpr (H == 2)
    asm volatile("v_fmac_f32_dpp %0, %0, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf" : "+v"(x) : "v"(s));
  else
    asm volatile("v_fmac_f32_dpp %0, %0, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf" : "+v"(x) : "v"(s));
}
template <int R>
__device__ __forceinline__ void dpp_enter(float2 (&v)[R]) {
#pragma unroll
  for (int m = 0; m < R; ++m) asm volatile("" : "+v"(v[m].x), "+v"(v[m].y));
  asm volatile("s_nop 1");
}
template <int R>
__device__ __forceinline__ void dpp_leave(float2 (&v)[R]) {
  asm volatile("s_nop 1");
#pragma unroll
  for (int m = 0; m < R; ++m) asm volatile("" : "+v"(v[m].x), "+v"(v[m].y));
}
// v[m] <- v[m] + s * partner(v[m]) for every register: for the lanes of the
// top half of each pair (s = 1) the butterfly output p + v, for the bottom
// half (s = -1) its negation -(p - v); rounding is symmetric under
// negation, so the caller recovers the output bit for bit by multiplying
// with s, which it folds into the next twiddle.
template <int L, int H, int R>
__device__ __forceinline__ void butterfly_fused(float2 (&v)[R], float s) {
  dpp_enter(v);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    dpp_fmac<L, H>(v[m].x, s);
    dpp_fmac<L, H>(v[m].y, s);
  }
  dpp_leave(v);
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
__host__ __device__ constexpr int bitrev_n(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r = (r << 1) | ((x >> i) & 1);
  return r;
}

// ----------------------------------------------------------------------------
// Tile configuration
// ----------------------------------------------------------------------------
// N: field size; L: lanes per line; K: workgroups sharing one field.
// With K == 1 the whole field is in one workgroup and transposes go
// through LDS; with K > 1 workgroup `part` owns lines [part*N/K, ...) in
// both layouts and transposes go through an L2-resident exchange buffer.
template <int N_, int L_, int K_ = 1>
struct TileCfg {
  static constexpr int N = N_;
  static constexpr int L = L_;
  static constexpr int K = K_;
  static constexpr int R = N / L;
  static constexpr int RPW = 64 / L;            // lines per wave
  static constexpr int LINES = N / K;           // lines per workgroup
  static constexpr int WAVES = LINES / RPW;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int LOGL = ilog2(L);
  static constexpr int PITCH = N + 8;           // LDS row pitch in float2 (bank spread)
  // LDS field buffer: the transpose buffer (K == 1), else one row per own
  // line for the propagation's stash.
  static constexpr int LDS_FIELD = (K == 1 ? N : LINES) * PITCH;
  // Registers per lane: a SIMD holds 512 per lane, shared by the waves of
  // the workgroup that land on it (waves are spread over the 4 SIMDs).
  static constexpr int WAVES_PER_SIMD = (WAVES + 3) / 4;
  static constexpr int REGS = 512 / WAVES_PER_SIMD;
  // With 256 or fewer registers the scheduler is fenced so that table loads
  // are not hoisted early (they spill otherwise); tiles with the full 512
  // registers and up to 16 values per lane, or 256 registers and up to 12,
  // also prefetch the next slice's chunk.
  static constexpr bool FENCE = REGS <= 256;
  static constexpr bool PREFETCH = (REGS >= 512 && R <= 16) || (REGS >= 256 && R <= 12);
  static_assert(N % L == 0 && LINES % RPW == 0 && WAVES >= 1, "bad tile");
};

// Per-thread coordinates.
template <class C>
struct Lane {
  int tid, w, g, l, q, k1, line;
  __device__ __forceinline__ explicit Lane(int t, int part = 0) {
    tid = t;
    w = t >> 6;
    int lane = t & 63;
    g = lane / C::L;
    l = lane % C::L;
    // logical index of the lane: the DPP partner of every radix-2 span is
    // the lane holding logical index q ^ span (L = 8: lanes 4..7 hold 7..4;
    // L = 16: lanes 8..15 hold the L = 8 order of lanes 7..0, plus 8)
    const int l8 = C::L == 16 && l >= 8 ? 15 - l : l;
    const int q8 = (C::L >= 8 && l8 >= 4) ? 11 - l8 : l8;
    q = (C::L == 16 && l >= 8) ? (q8 ^ 8) : q8;
    k1 = bitrev_n(q, C::LOGL);
    line = part * C::LINES + w * C::RPW + g;
  }
  __device__ __forceinline__ int pos_nat(int m) const { return q + C::L * m; }
  __device__ __forceinline__ int pos_spec(int m) const { return C::R * k1 + m; }
  __device__ __forceinline__ int pos(int m, bool spec) const { return spec ? pos_spec(m) : pos_nat(m); }
};

// Shared tables (LDS), forward sign, built in FP64 and rounded once.
template <class C>
struct Tables {
  float2 wn[C::N];          // W_N^e = exp(-2 pi i e / N), e in [0, N)
  float2 tw[C::R * C::L];   // entry k2*L + q: W_N^{q k2} (inter-stage twiddles)
  float2 h[C::N];           // (1D Fresnel kernel - 1) / N at spectral slot m*L + k1 (frequency R*k1 + m)
};

template <class C>
__device__ void build_twiddles(Tables<C>& tb, int tid) {
  for (int e = tid; e < C::N; e += C::THREADS) {
    double s, c;
    sincospi(-2.0 * double(e) / double(C::N), &s, &c);
    tb.wn[e] = make_float2(float(c), float(s));
  }
  for (int i = tid; i < C::R * C::L; i += C::THREADS) {
    const int k2 = i / C::L, q = i % C::L;
    double s, c;
    sincospi(-2.0 * double((q * k2) % C::N) / double(C::N), &s, &c);
    tb.tw[i] = make_float2(float(c), float(s));
  }
}

// 1D Fresnel kernel minus one, (exp(i pi (lambda dz / dx^2) f^2) - 1) / N,
// f = fftfreq(N), stored so that the L lanes of a line read L consecutive
// entries.  The real part is -2 sin^2(theta/2), exact for small phases.
template <class C>
__device__ void build_fresnel(Tables<C>& tb, int tid, double chirp /* lambda dz / dx^2 */) {
  for (int idx = tid; idx < C::N; idx += C::THREADS) {
    const int m = idx / C::L, k1 = idx % C::L;
    const int k = C::R * k1 + m;
    int kk = (k < (C::N + 1) / 2) ? k : k - C::N;
    double f = double(kk) / double(C::N);
    const double x = chirp * f * f;          // phase / pi
    const double sh = sinpi(0.5 * x);
    // the lane holding slot k1 has logical index q = bitrev(k1); with the
    // forward transform's last stage fused its output there is negated
    // when q is odd (propagate_line), so the table holds the negated kernel
    const double sg = (ADORYM_FUSED_DPP && (bitrev_n(k1, C::LOGL) & 1)) ? -1.0 : 1.0;
    tb.h[idx] = make_float2(float(sg * -2.0 * sh * sh / C::N), float(sg * sinpi(x) / C::N));
  }
}

// W_N^{SIGN * e} for 0 <= e < N.
template <class C, int SIGN>
__device__ __forceinline__ float2 wn_at(const Tables<C>& tb, int e) {
  float2 w = tb.wn[e];
  return SIGN < 0 ? w : cconj(w);
}
// W_N^{SIGN * q * k2} for the thread's lane index q.
template <class C, int SIGN>
__device__ __forceinline__ float2 tw_at(const Tables<C>& tb, int q, int k2) {
  float2 w = tb.tw[k2 * C::L + q];
  return SIGN < 0 ? w : cconj(w);
}

// Scheduling fence: keeps the scheduler from hoisting table loads of later
// groups (the tile is register-bound at 1024 threads per workgroup).
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

template <class C, int SIGN>
__device__ __forceinline__ void apply_twiddles(float2 (&v)[C::R], const Tables<C>& tb, const Lane<C>& ln) {
#pragma unroll
  for (int k2 = 1; k2 < C::R; ++k2) {
    v[k2] = cmul(v[k2], tw_at<C, SIGN>(tb, ln.q, k2));
    if (C::FENCE && (k2 & 3) == 3) sched_fence();
  }
  if (C::FENCE) sched_fence();
}

// ----------------------------------------------------------------------------
// 1D DFT along the thread's line: natural order -> spectral order.
// SIGN = -1: forward DFT (exp(-...)), +1: inverse (unnormalised).
// ----------------------------------------------------------------------------
// SIGNED_OUT: the last stage (span 1) is fused too and the lanes with q odd
// return the negated output (lane_sign_fft); the caller folds that sign
// into what it multiplies the spectrum by.
template <class C, int SIGN, bool SIGNED_OUT = false>
__device__ __forceinline__ void fft_line(float2 (&v)[C::R], const Tables<C>& tb, const Lane<C>& ln) {
  Dft<C::R, SIGN, 1, 0, C::R>::run(v);
  // twiddle W_N^{q k2}
  apply_twiddles<C, SIGN>(v, tb, ln);
  // cross-lane DIF, spans L/2 ... 1
  CFor<0, C::LOGL>::run([&](auto sc) {
    constexpr int H = C::L >> (decltype(sc)::value + 1);
    const bool top = (ln.q & H) == 0;
    const float sgn = top ? 1.f : -1.f;
    // bottom lanes of a pair take W_{2H}^{q mod H}; top lanes W^0 = 1
    const float2 wl = wn_at<C, SIGN>(tb, top ? 0 : (ln.q & (H - 1)) * (C::N / (2 * H)));
    if constexpr (ADORYM_FUSED_DPP && H == 1 && SIGNED_OUT) {
      butterfly_fused<C::L, H>(v, sgn);        // sgn (p + sgn v); no twiddle at span 1
    } else if constexpr (ADORYM_FUSED_DPP && H > 1) {
      // sgn (p + sgn v) in one fused op per value; sgn goes into the twiddle
      butterfly_fused<C::L, H>(v, sgn);
      const float2 ws = make_float2(sgn * wl.x, sgn * wl.y);
#pragma unroll
      for (int m = 0; m < C::R; ++m) v[m] = cmul(v[m], ws);
    } else {
#pragma unroll
      for (int m = 0; m < C::R; ++m) {
        float2 p = partner<C::L, H>(v[m]);
        float2 d = make_float2(p.x + sgn * v[m].x, p.y + sgn * v[m].y);
        if constexpr (H > 1) d = cmul(d, wl);
        v[m] = d;
      }
    }
  });
}

// 1D DFT along the line: spectral order -> natural order.  SIGNED_OUT: the
// last stage (span L/2) is fused too, and the lanes with q & L/2 return the
// negated output (lane_sign_ifft): every later operation is linear in the
// lane's values, and rounding is symmetric under negation, so the sign comes
// out unchanged for the caller to take back.
template <class C, int SIGN, bool SIGNED_OUT = false>
__device__ __forceinline__ void ifft_line(float2 (&v)[C::R], const Tables<C>& tb, const Lane<C>& ln) {
  // cross-lane DIT, spans 1 ... L/2 (bit-reversed in, natural out).  The
  // fused stages (all but the last) leave their output times the lane's
  // sign `carry`, which the next stage's twiddle takes back.
  float carry = 1.f;
  CFor<0, C::LOGL>::run([&](auto sc) {
    constexpr int H = 1 << decltype(sc)::value;
    const bool top = (ln.q & H) == 0;
    const float sgn = top ? 1.f : -1.f;
    float2 wl = wn_at<C, SIGN>(tb, top ? 0 : (ln.q & (H - 1)) * (C::N / (2 * H)));
    if constexpr (ADORYM_FUSED_DPP && H > 1) wl = make_float2(carry * wl.x, carry * wl.y);
    if constexpr (ADORYM_FUSED_DPP && (2 * H < C::L || SIGNED_OUT)) {
      if constexpr (H > 1) {
#pragma unroll
        for (int m = 0; m < C::R; ++m) v[m] = cmul(v[m], wl);
      }
      butterfly_fused<C::L, H>(v, sgn);
      carry = sgn;
    } else {
#pragma unroll
      for (int m = 0; m < C::R; ++m) {
        float2 u = v[m];
        if constexpr (H > 1) u = cmul(u, wl);
        float2 p = partner<C::L, H>(u);
        v[m] = make_float2(p.x + sgn * u.x, p.y + sgn * u.y);
      }
    }
  });
  apply_twiddles<C, SIGN>(v, tb, ln);
  Dft<C::R, SIGN, 1, 0, C::R>::run(v);
}

// Fresnel propagation along the line (CONJ: adjoint kernel), written as
// v + IDFT((h - 1) DFT(v)) / N: the transforms carry only the small change
// the propagation makes (|h - 1| is about 1e-2 for these distances), so
// their float32 rounding is relative to that change rather than to the wave.
// K == 1 tiles keep the input in the thread's own cells of the LDS transpose
// buffer (stash: the line's row) instead of registers.
// The transforms run with both last stages fused (SIGNED_OUT): the Fresnel
// table already holds each slot's kernel times the sign the forward
// transform leaves on its lane (build_fresnel), so the product is exact,
// and the inverse transform's lane sign is taken back in the final sum.
template <class C, bool CONJ>
__device__ __forceinline__ void propagate_line(float2 (&v)[C::R], const Tables<C>& tb, const Lane<C>& ln,
                                               float2* stash = nullptr) {
  constexpr bool SGN = ADORYM_FUSED_DPP;
  float2 v0[C::R];
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    if (stash) stash[ln.pos_nat(m)] = v[m];
    else v0[m] = v[m];
  }
  fft_line<C, -1, SGN>(v, tb, ln);
  if (C::FENCE) sched_fence();
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    float2 h = tb.h[m * C::L + ln.k1];     // kernel - 1 at frequency R*k1 + m (times the lane sign)
    v[m] = CONJ ? cmulc(v[m], h) : cmul(v[m], h);
    if (C::FENCE && (m & 3) == 3) sched_fence();
  }
  ifft_line<C, +1, SGN>(v, tb, ln);
  const float so = SGN && (ln.q & (C::L / 2)) ? -1.f : 1.f;
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const float2 u = stash ? stash[ln.pos_nat(m)] : v0[m];
    v[m] = make_float2(fmaf(so, v[m].x, u.x), fmaf(so, v[m].y, u.y));
  }
}

// ----------------------------------------------------------------------------
// Transpose through LDS: the thread's line layout flips (ROW <-> COL).
// src_spec / dst_spec: whether the along-line positions are in spectral
// order before / after.  Line indices are always natural.
// ----------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ void transpose(float2 (&v)[C::R], float2* buf, const Lane<C>& ln,
                                          bool src_spec, bool dst_spec) {
  __syncthreads();
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    int a = ln.line, b = ln.pos(m, src_spec);       // (line, pos) in source layout
    buf[a * C::PITCH + b] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    int a = ln.pos(m, dst_spec), b = ln.line;       // destination line = source pos
    v[m] = buf[a * C::PITCH + b];
  }
}

// ----------------------------------------------------------------------------
// Raw buffer access with 32-bit byte offsets (one VGPR offset per thread,
// uniform strides in SGPRs).  Accesses at or beyond `bytes` read 0 / are
// dropped by the hardware range check.
// ----------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit buffer, gfx9 family

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// Two-float buffer access through the LLVM intrinsics directly (the b64
// clang builtin lowers to a single dword load on this toolchain).
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ f32x2 adorym_raw_load_v2f32(rsrc_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.ptr.buffer.load.v2f32");
__device__ void adorym_raw_store_v2f32(f32x2 v, rsrc_t rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.ptr.buffer.store.v2f32");

// Cache-policy operand: 0 = default; kCoherent = sc0|sc1 (system scope:
// stores write through every cache level, loads miss in every cache), used
// for data that other workgroups read within the same kernel.
constexpr int kCoherent = 1 | 16;
// nt: streaming data, a hint to keep it from displacing reused lines.
constexpr int kNonTemporal = 2;

template <int AUX = 0>
__device__ __forceinline__ float2 bload2(rsrc_t r, uint32_t voff, uint32_t soff) {
  const f32x2 t = adorym_raw_load_v2f32(r, (int)voff, (int)soff, AUX);
  return make_float2(t.x, t.y);
}
template <int AUX = 0>
__device__ __forceinline__ void bstore2(rsrc_t r, float2 v, uint32_t voff, uint32_t soff) {
  f32x2 t;
  t.x = v.x;
  t.y = v.y;
  adorym_raw_store_v2f32(t, r, (int)voff, (int)soff, AUX);
}
__device__ __forceinline__ void batomic_add(rsrc_t r, float v, uint32_t voff, uint32_t soff) {
  (void)__builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(v, r, voff, soff, 0);
}

// ----------------------------------------------------------------------------
// Cross-workgroup exchange (K > 1)
// ----------------------------------------------------------------------------
// The K workgroups of a field meet at a barrier on a per-field counter.  The
// counter only grows: the t-th barrier waits for K*t arrivals.  No
// device-scope fences are used (on this chip they write back and invalidate
// the per-XCD L2 caches): the exchanged data bypasses the caches
// (kCoherent), each wave waits for its own stores to complete before the
// workgroup barrier, and the counter is read and updated with relaxed
// device-scope atomics.  The wait is bounded so that a group that cannot be
// co-resident sets an error bit and finishes instead of hanging.
constexpr int kSpinLimit = 1 << 22;
constexpr int kErrBarrierTimeout = 2;

__device__ __forceinline__ void wait_stores() {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's memory operations have completed
}

// The barrier in two halves, so that work that touches no exchanged data can
// run between the arrival and the wait.  The arrival returns (in thread 0)
// whether it was the last one the barrier waits for: that workgroup need
// not poll the counter at all.
__device__ __forceinline__ bool group_arrive(int* counter, int target) {
  wait_stores();
  __syncthreads();
  bool last = false;
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 >= target;
  return last;
}
__device__ __forceinline__ void group_wait(int* counter, int target, int* err, bool last) {
  if (threadIdx.x == 0 && !last) {
    int spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        __hip_atomic_fetch_or(err, kErrBarrierTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}
__device__ __forceinline__ void group_barrier(int* counter, int target, int* err) {
  group_wait(counter, target, err, group_arrive(counter, target));
}

// Exchange state of one field group: two alternating N x N halves per field
// slot, the barrier counter and the number of barriers passed so far.
// `local` is set when every member of the group runs on the same XCD: the
// exchange then stays in that XCD's L2 (stores write through the L1, loads
// skip it); otherwise it goes through memory (kCoherent).
struct Exchange {
  float2* buf;      // [2 phases][2 fields][N][N]
  int* counter;
  int* err;
  int phase;
  bool local;
  bool last;        // split-phase transpose: this workgroup's arrival completed the barrier
};

constexpr int kL1Bypass = 1;      // sc0: load misses in the L1, hits in L2

__device__ __forceinline__ int xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);   // HW_REG_XCC_ID bits [3:0]
}

// First barrier of a group: publish this workgroup's XCD, learn whether all
// members share one.  ids: [K] ints of this field's group.
template <int K>
__device__ __forceinline__ void exchange_init(Exchange& x, int* ids, int part) {
  x.phase = 0;
  x.local = false;
  if (threadIdx.x == 0) __hip_atomic_store(ids + part, xcc_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  ++x.phase;
  group_barrier(x.counter, K * x.phase, x.err);
  bool same = true;
  const int first = __hip_atomic_load(ids, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int i = 1; i < K; ++i) same &= __hip_atomic_load(ids + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == first;
  x.local = same;
}

template <class C, int NF, int LD, int ST>
__device__ __forceinline__ void transpose_global_impl(float2 (&v0)[C::R], float2 (&v1)[C::R], Exchange& x,
                                                      const Lane<C>& ln, bool src_spec, bool dst_spec) {
  constexpr int NN = C::N * C::N;
  float2* base = x.buf + (size_t)(x.phase & 1) * 2 * NN;
  const rsrc_t r = make_rsrc(base, 2 * NN * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const uint32_t off = (uint32_t)(ln.line * C::N + ln.pos(m, src_spec)) * 8;
    bstore2<ST>(r, v0[m], off, 0);
    if (NF == 2) bstore2<ST>(r, v1[m], off, NN * 8);
  }
  ++x.phase;
  group_barrier(x.counter, C::K * x.phase, x.err);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const uint32_t off = (uint32_t)(ln.pos(m, dst_spec) * C::N + ln.line) * 8;
    v0[m] = bload2<LD>(r, off, 0);
    if (NF == 2) v1[m] = bload2<LD>(r, off, NN * 8);
  }
}

// Transpose of one or two fields through the exchange buffer (K > 1).
template <class C, int NF>
__device__ __forceinline__ void transpose_global(float2 (&v0)[C::R], float2 (&v1)[C::R], Exchange& x,
                                                 const Lane<C>& ln, bool src_spec, bool dst_spec) {
  if (x.local) transpose_global_impl<C, NF, kL1Bypass, 0>(v0, v1, x, ln, src_spec, dst_spec);
  else transpose_global_impl<C, NF, kCoherent, kCoherent>(v0, v1, x, ln, src_spec, dst_spec);
}

// The same transpose in two halves: begin stores this workgroup's lines and
// arrives at the group barrier; end waits and loads the transposed lines.
// Between the two the caller may do work that touches neither field.
template <class C, int NF, int ST>
__device__ __forceinline__ void transpose_begin_impl(const float2 (&v0)[C::R], const float2 (&v1)[C::R], Exchange& x,
                                                     const Lane<C>& ln, bool src_spec) {
  constexpr int NN = C::N * C::N;
  const rsrc_t r = make_rsrc(x.buf + (size_t)(x.phase & 1) * 2 * NN, 2 * NN * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const uint32_t off = (uint32_t)(ln.line * C::N + ln.pos(m, src_spec)) * 8;
    bstore2<ST>(r, v0[m], off, 0);
    if (NF == 2) bstore2<ST>(r, v1[m], off, NN * 8);
  }
  ++x.phase;
  x.last = group_arrive(x.counter, C::K * x.phase);
}
template <class C, int NF, int LD>
__device__ __forceinline__ void transpose_end_impl(float2 (&v0)[C::R], float2 (&v1)[C::R], Exchange& x,
                                                   const Lane<C>& ln, bool dst_spec) {
  constexpr int NN = C::N * C::N;
  group_wait(x.counter, C::K * x.phase, x.err, x.last);
  const rsrc_t r = make_rsrc(x.buf + (size_t)((x.phase - 1) & 1) * 2 * NN, 2 * NN * 8);
#pragma unroll
  for (int m = 0; m < C::R; ++m) {
    const uint32_t off = (uint32_t)(ln.pos(m, dst_spec) * C::N + ln.line) * 8;
    v0[m] = bload2<LD>(r, off, 0);
    if (NF == 2) v1[m] = bload2<LD>(r, off, NN * 8);
  }
}
template <class C, int NF>
__device__ __forceinline__ void transpose_global_begin(const float2 (&v0)[C::R], const float2 (&v1)[C::R],
                                                       Exchange& x, const Lane<C>& ln, bool src_spec) {
  if (x.local) transpose_begin_impl<C, NF, 0>(v0, v1, x, ln, src_spec);
  else transpose_begin_impl<C, NF, kCoherent>(v0, v1, x, ln, src_spec);
}
template <class C, int NF>
__device__ __forceinline__ void transpose_global_end(float2 (&v0)[C::R], float2 (&v1)[C::R], Exchange& x,
                                                     const Lane<C>& ln, bool dst_spec) {
  if (x.local) transpose_end_impl<C, NF, kL1Bypass>(v0, v1, x, ln, dst_spec);
  else transpose_end_impl<C, NF, kCoherent>(v0, v1, x, ln, dst_spec);
}

// ----------------------------------------------------------------------------
// Block reductions
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <int THREADS>
__device__ __forceinline__ double block_sum(double x, double* scratch /* >= THREADS/64 */) {
  x = wave_sum(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) scratch[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < THREADS / 64; ++i) r += scratch[i];   // fixed order
  }
  return r;  // valid in thread 0 only
}

}  // namespace adorym
