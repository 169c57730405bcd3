// Device building blocks of the affine-arithmetic bound (gfx950).
//
// One wavefront owns BPW = 256/H boxes.  A box's affine form (Appendix A:
// center x0, generator matrix X, condensed term xinf) lives in an LDS tile of
// NS = 16*NT term slots (slot 0 = center, slots 1.. = noise-symbol columns)
// by H rows.  Two register layouts alternate:
//
//  * MFMA layout: each hidden linear layer [y0|Y] = W [x0|X] (Table 2 matrix
//    multiplication) is a 16x16x4 FP32 MFMA GEMM; lane (g,c) = (lane/16,
//    lane%16) holds accumulator rows 16t+4g+j of column c.
//  * owner layout: lane l owns 4 complete rows (row slots 4l..4l+3) with all
//    their NS terms, so the per-neuron work of the activation (Table 3
//    linearisation, eq. affine_func_update) is lane-local, and only the
//    column reductions of truncation (Section 3.3) cross lanes.
//
// In the rigorous mode (the default) every floating-point rounding (MFMA
// accumulation, FP64 center, activation parameters, transcendental
// functions, condensation sums) is bounded a priori and folded into the
// condensed coefficient, a per-neuron error symbol, so the form encloses the
// exact network at every layer and the final [lo, hi] is a sound enclosure
// although the arithmetic is FP32.  Without it the arithmetic is the
// paper's, which the parity tests compare with the FP64 oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "spk_impl.h"

namespace spk {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr float kU = 5.9604644775390625e-08f;    // 2^-24, unit roundoff of binary32
constexpr float kEta = 7.8886090522101181e-31f;  // 2^-100, absolute slack (underflow, flushes)
constexpr float kGrow = 1.0f + 9.5367431640625e-07f;   // 1 + 2^-20
constexpr float kGrowR = 1.0f + 1.52587890625e-05f;    // 1 + 2^-16
constexpr float kTwoPi = 6.28318548202514648f;    // binary32 nearest to 2 pi
constexpr float kInvTwoPi = 0.159154936671257019f;
constexpr float kPi = 3.14159274101257324f;

__device__ __forceinline__ float next_up(float x) {
  if (!(x < INFINITY)) return x;  // +inf or NaN
  if (x == 0.0f) return 1.17549435e-38f;
  uint32_t u = __float_as_uint(x);
  u = (x > 0.0f) ? u + 1u : u - 1u;
  return __uint_as_float(u);
}

__device__ __forceinline__ float next_down(float x) { return -next_up(-x); }

template <int H_, int NT_>
struct Shape {
  static constexpr int H = H_;
  static constexpr int MT = H / 16;              // 16-row tiles per box
  static constexpr int NT = NT_;                 // 16-column tiles per box
  static constexpr int NS = 16 * NT;             // term slots per box
  static constexpr int BPW = 256 / H;            // boxes per wavefront
  static constexpr int SEG = H / 4;              // owner lanes per box
  static constexpr int TILE = BPW * NS * H;      // floats of the LDS tile
  static constexpr int SWM = ((H / 4) < 16 ? (H / 4) : 16) - 1;
};

// Float index of the 4-row chunk `ch` (rows 4ch..4ch+3) of term slot C of box
// b in the tile.  Chunks are XOR-swizzled with the slot index so that both
// the MFMA-layout stores and the owner-layout loads spread over the banks.
template <class S>
__device__ __forceinline__ int taddr(int b, int C, int ch) {
  return (b * S::NS + C) * S::H + ((ch ^ (C & S::SWM)) << 2);
}

template <int SEG>
__device__ __forceinline__ float seg_allsum(float v) {
#pragma unroll
  for (int m = 1; m < SEG; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Number of lanes of this lane's segment (SEG consecutive lanes) with p set.
template <int SEG>
__device__ __forceinline__ unsigned long long seg_mask(int lane) {
  if constexpr (SEG == 64) {
    return ~0ull;
  } else {
    return ((1ull << SEG) - 1ull) << ((lane / SEG) * SEG);
  }
}

template <int SEG>
__device__ __forceinline__ int seg_count(bool p, int lane) {
  const unsigned long long m = __ballot(p);
  return __popcll(m & seg_mask<SEG>(lane));
}

// Same, restricted to the lanes of the segment below this lane.
template <int SEG>
__device__ __forceinline__ int seg_count_below(bool p, int lane) {
  const unsigned long long m = __ballot(p);
  const unsigned long long below = (1ull << lane) - 1ull;
  return __popcll(m & below & seg_mask<SEG>(lane));
}

// Position of the n-th (0-based) set bit of m (m must have more than n set bits).
__device__ __forceinline__ int nth_set_bit(uint32_t m, int n) {
  int pos = 0;
#pragma unroll
  for (int w = 16; w >= 1; w >>= 1) {
    const uint32_t low = m & ((1u << w) - 1u);
    const int cnt = __popc(low);
    const bool up = n >= cnt;
    n = up ? n - cnt : n;
    m = up ? (m >> w) : low;
    pos += up ? w : 0;
  }
  return pos;
}

// ---------------------------------------------------------------------------
// Linearisation parameters (Table 3), computed in FP64 from the FP64 range
// [xl, xu].  `dg` bounds how much the true maximum error of alpha*x + beta on
// [xl, xu] can exceed the returned gamma (evaluation rounding and the ulp
// error of the transcendental functions).  FP64 matters here: for narrow
// ranges gamma is a difference of nearly equal numbers (ELU, sin), which
// loses ~1e-3 of the bound in FP32 on 8-layer networks.
// ---------------------------------------------------------------------------
struct ActOut {
  double al, be, ga;
  float dg;
};

constexpr double kUd = 1.1102230246251565e-16;   // 2^-53

template <int ACT>
__device__ __forceinline__ ActOut act_params(double xl, double xu, double x0);

template <>
__device__ __forceinline__ ActOut act_params<SPK_ACT_RELU>(double xl, double xu, double x0) {
  ActOut o;
  if (xl >= 0.0) {
    o.al = 1.0; o.be = 0.0; o.ga = 0.0; o.dg = 0.0f;
  } else if (xu <= 0.0) {
    o.al = 0.0; o.be = 0.0; o.ga = 0.0; o.dg = 0.0f;
  } else {
    // chord slope; beta = (ReLU(xl) - alpha xl)/2; the maximum error equals beta
    o.al = xu / (xu - xl);
    o.be = -0.5 * o.al * xl;
    o.ga = o.be;
    o.dg = (float)(8.0 * kUd * (xu - xl));
  }
  return o;
}

__device__ __forceinline__ double elu_d(double x) { return x > 0.0 ? x : expm1(x); }

template <>
__device__ __forceinline__ ActOut act_params<SPK_ACT_ELU>(double xl, double xu, double x0) {
  ActOut o;
  if (xl >= 0.0) {
    o.al = 1.0; o.be = 0.0; o.ga = 0.0; o.dg = 0.0f;
    return o;
  }
  const double w = xu - xl;
  double al;
  if (xu <= 0.0) {
    // chord of e^x - 1 on [xl, xu] without cancellation: e^xl (e^w - 1)/w
    al = (w > 0.0) ? exp(xl) * (expm1(w) / w) : exp(xl);
  } else {
    al = (xu - expm1(xl)) / w;
  }
  al = fmin(fmax(al, 1.0e-300), 1.0);
  // upper error at the interval ends; lower error at the tangent point ln(alpha)
  const double ru = fmax(elu_d(xl) - al * xl, elu_d(xu) - al * xu);
  const double rl = (al - 1.0) - al * log(al);
  o.al = al;
  o.be = 0.5 * (ru + rl);
  o.ga = ru - o.be;
  o.dg = (float)(32.0 * kUd * (fabs(xl) + fabs(xu) + 1.0));
  return o;
}

template <>
__device__ __forceinline__ ActOut act_params<SPK_ACT_SIN>(double xl, double xu, double x0) {
  const double twopi = 6.283185307179586, inv = 0.15915494309189535, pi = 3.141592653589793;
  ActOut o;
  // range of cos on [xl, xu]: end values, widened to +-1 when a maximum
  // (2 pi j) or minimum (pi + 2 pi j) lies inside
  const double cl = cos(xl), cu = cos(xu);
  double slo = fmin(cl, cu), shi = fmax(cl, cu);
  if (ceil(xl * inv) * twopi <= xu) shi = 1.0;
  if (ceil((xl - pi) * inv) * twopi + pi <= xu) slo = -1.0;
  double al = 0.5 * (slo + shi);
  al = fmin(fmax(al, -1.0), 1.0);
  const double ep = acos(al);
  // candidates: ends, first and last stationary point of each family +-ep + 2 pi j
  double cand[6];
  cand[0] = xl;
  cand[1] = xu;
  cand[2] = ceil((xl + ep) * inv) * twopi - ep;
  cand[3] = ceil((xl - ep) * inv) * twopi + ep;
  cand[4] = floor((xu - ep) * inv) * twopi + ep;
  cand[5] = floor((xu + ep) * inv) * twopi - ep;
  double ru = -INFINITY, rl = INFINITY;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double x = fmin(fmax(cand[q], xl), xu);
    const double v = sin(x) - al * x;
    ru = fmax(ru, v);
    rl = fmin(rl, v);
  }
  o.al = al;
  o.be = 0.5 * (ru + rl);
  o.ga = ru - o.be;
  const double M = fabs(xl) + fabs(xu) + 16.0;
  const double dx = 8.0 * kUd * M;
  o.dg = (float)(32.0 * kUd * (1.0 + fabs(al) * M + fabs(o.be)) + dx * dx) + kEta;
  return o;
}

}  // namespace spk
