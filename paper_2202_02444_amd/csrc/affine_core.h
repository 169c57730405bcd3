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

// Cross-lane sums on the VALU: DPP moves inside a 16-lane row and the gfx950
// row-swap instructions between rows, instead of LDS permutes (each of which
// the compiler waits for before the next one).  Lane groups of 2^m lanes are
// combined pairwise exactly as by an XOR butterfly over the masks 1, 2, ...,
// so every lane of a segment holds the same bits, and the same bits as the
// butterfly.  DPP controls: quad_perm [1,0,3,2] and [2,3,0,1] pair lanes
// c ^ 1 and c ^ 2; once quads (halves of a row) hold one value each, the
// half-row mirror (c -> 7 - c) and the row mirror (c -> 15 - c) pair the two
// quads of each half and the two halves of each row.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __uint_as_float(dpp_u32<CTRL>(__float_as_uint(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = dpp_u32<CTRL>((uint32_t)u), hi = dpp_u32<CTRL>((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(lo | (hi << 32)));
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppRowMirror = 0x140, kDppHalfMirror = 0x141;

// The values of this lane's partner row (rows 2r and 2r+1 of 16 lanes pair up)
// and partner half (lanes l and l ^ 32), from v_permlane16_swap_b32 and
// v_permlane32_swap_b32 with both operands v: one returned operand holds the
// even row's (lower half's) value and the other the odd row's (upper half's),
// in every lane of the pair, so their sum is the same in both.
__device__ __forceinline__ float row_pair_sum(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float half_pair_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double row_pair_sum(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
  return __longlong_as_double((long long)((uint64_t)l[0] | ((uint64_t)h[0] << 32))) +
         __longlong_as_double((long long)((uint64_t)l[1] | ((uint64_t)h[1] << 32)));
}
__device__ __forceinline__ double half_pair_sum(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane32_swap((uint32_t)u, (uint32_t)u, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
  return __longlong_as_double((long long)((uint64_t)l[0] | ((uint64_t)h[0] << 32))) +
         __longlong_as_double((long long)((uint64_t)l[1] | ((uint64_t)h[1] << 32)));
}

// Sum over the SEG consecutive lanes of this lane's segment (SEG = 8, 16, 32
// or 64), the same value in every lane of it.
template <int SEG, class T>
__device__ __forceinline__ T seg_allsum_t(T v) {
  static_assert(SEG == 8 || SEG == 16 || SEG == 32 || SEG == 64, "segments of 8 to 64 lanes");
  if constexpr (sizeof(T) == 4) {
    v += dpp_f<kDppXor1>(v);
    v += dpp_f<kDppXor2>(v);
    v += dpp_f<kDppHalfMirror>(v);
    if constexpr (SEG >= 16) v += dpp_f<kDppRowMirror>(v);
  } else {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    if constexpr (SEG >= 16) v += dpp_d<kDppRowMirror>(v);
  }
  if constexpr (SEG >= 32) v = row_pair_sum(v);
  if constexpr (SEG == 64) v = half_pair_sum(v);
  return v;
}
template <int SEG>
__device__ __forceinline__ float seg_allsum(float v) {
  return seg_allsum_t<SEG, float>(v);
}

// Sum over the four 16-lane rows (lanes l, l ^ 16, l ^ 32, l ^ 48).
template <class T>
__device__ __forceinline__ T rows_allsum(T v) {
  return half_pair_sum(row_pair_sum(v));
}
__device__ __forceinline__ float rows_allmax(float v) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
  r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
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
