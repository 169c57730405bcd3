// The affine-arithmetic network pass shared by the bound and ray kernels.
//
// A wavefront owns BPW boxes (or ray segments).  The steps:
//   activate()      activation linearisation + condensation, owner layout
//                   (eq. affine_func_update, Table 3, Section 3.3)
//   hidden_layer()  one H -> H layer: generators Y = W X on FP32 MFMA, the
//                   center W x0 in FP64, |W| xinf and the rounding-error
//                   product |W| u on VALU alongside (Table 2 matrix
//                   multiplication)
//   output_layer()  the H -> 1 layer and the range read-off (eq. def_range)
//
// "Passenger" slots (the last NPASS term slots) carry plain point
// evaluations through the same GEMMs: they receive the bias and the exact
// activation instead of the linearisation, and are excluded from the radius.
// The ray-march kernel uses them for the convergence test of Procedure 2.
#pragma once

#include "affine_core.h"

namespace spk {

constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53

template <class S>
struct LdsState {
  float tile[S::TILE];
  float vinf[256];
  double vc[256];
};

template <int ACT>
__device__ __forceinline__ float act_point(float x, float omega0) {
  if (ACT == SPK_ACT_RELU) return fmaxf(x, 0.0f);
  if (ACT == SPK_ACT_ELU) return x > 0.0f ? x : expm1f(x);
  return sinf(omega0 * x);
}

template <int SEG>
__device__ __forceinline__ double seg_allsum_d(double v) {
  return seg_allsum_t<SEG, double>(v);
}

// Round a double to a float that is <= / >= it.
__device__ __forceinline__ float round_down_f(double v) {
  float f = (float)v;
  return ((double)f > v) ? next_down(f) : f;
}
__device__ __forceinline__ float round_up_f(double v) {
  float f = (float)v;
  return ((double)f < v) ? next_up(f) : f;
}

// Activation + condensation on the owner-layout rows.  On entry xc holds the
// pre-activation centers (FP64, bias included), y the generator terms in
// slots 1.. (slot 0 is unused) and yinf the condensed term.  On exit
// xc/y/yinf hold the post-activation form.  Returns the new number of
// occupied generator slots.
//
// With rig = false this is the paper's arithmetic (rounding ignored, Section
// 3.4): the linearisation is taken on the computed range and e, u are not
// used.  With rig = true every floating-point rounding is bounded a priori and
// folded into the condensed term, which is itself a per-neuron error symbol
// (Appendix A), so the form stays a sound enclosure of the exact network:
//  * e (in) holds the errors created since the last fold (layer 0 input and
//    product rounding, bias addition, split-product absolute terms); it is
//    added to yinf first and cleared;
//  * the linearisation is taken on the range of the whole form, so it holds
//    wherever the exact pre-activation can lie;
//  * the rounding of alpha x0 + beta, of alpha Y, of alpha yinf, of gamma and
//    the evaluation error of (alpha, beta, gamma) go into yinf;
//  * condensed sums are rounded upwards;
//  * last, yinf receives u = cK r + cD |x0|, the a-priori rounding of the next
//    layer's products (generators in FP32, split precision or FP64 against W,
//    the center in FP64): that layer's |W| yinf then carries it; generators
//    produced in FP64 and stored in FP32 add uY times their stored magnitude
//    before the range is read off.
//
// With `sent` non-null (first activation of a bound pass, truncate), every
// kept new term placed in a slot C >= 4 is also recorded as the single entry
// of its column: sent[C] = its value gamma_j and sent[S::NS + C] = its row j
// (as an int), for the first hidden layer's row-owner products.
template <class S, int ACT, int POL, int NPASS>
__device__ __forceinline__ int activate(double (&xc)[4], f4 (&y)[S::NS], float (&yinf)[4], float (&e)[4],
                                        float (&u)[4], int n_occ, int k, float cK, float cD, float omega0, int lane,
                                        int16_t* rec, float* sent = nullptr, bool rig = false, float uY = 0.0f) {
  static_assert(NPASS == 0 || POL == SPK_AFFINE_FIXED, "passengers ride along affine-fixed passes only");
  constexpr int NG = S::NS - NPASS;   // slots 1..NG-1 are generators
  float gam[4], rnext[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int C = NG; C < S::NS; ++C) y[C][i] = act_point<ACT>(y[C][i], omega0);
    if (rig) {
      yinf[i] = round_up_f((double)yinf[i] + (double)e[i]);
      e[i] = 0.0f;
    }
    if (ACT == SPK_ACT_SIN) {
      // Table 2 constant multiplication by omega0 before sin
      float rs = 0.0f;
#pragma unroll
      for (int C = 1; C < NG; ++C) {
        y[C][i] *= omega0;
        rs += fabsf(y[C][i]);
      }
      xc[i] *= (double)omega0;
      if (rig) {
        // products by omega0 (FP32 generators and yinf, FP64 center)
        const double ys = (double)yinf[i] * (double)omega0;
        yinf[i] = round_up_f((ys + (double)kU * ((double)rs + ys)) * (1.0 + 4.0 * kU64) + 2.0 * kU64 * fabs(xc[i]) +
                             (double)kEta);
      } else {
        yinf[i] *= omega0;
      }
    }
    const double x0 = xc[i];
    // the range radius is summed in FP64: the linearisation parameters of a
    // narrow straddling neuron are sensitive to it
    double rYd = 0.0;
#pragma unroll
    for (int C = 1; C < NG; ++C) rYd += (double)fabsf(y[C][i]);
    // rigorous: generators produced in FP64 and stored in FP32 are within uY
    // of their stored magnitude; the range must cover the exact values
    if (rig && uY > 0.0f) yinf[i] = round_up_f((double)yinf[i] + (double)uY * rYd * (1.0 + (double)(NG + 2) * kU64));
    double rd = rYd + (double)yinf[i];
    // rigorous: an FP64 sum of NG terms is within (NG + 1) 2^-53 of exact
    if (rig) rd = rd * (1.0 + (double)(NG + 2) * kU64) + (double)kEta;
    const float rY = round_up_f(rYd);
    const float r = round_up_f(rd);
    const double xl = x0 - rd, xu = x0 + rd;
    const ActOut p = act_params<ACT>(xl, xu, x0);
    const float alf = (float)p.al;
    const double z0 = fma(p.al, x0, p.be);
#pragma unroll
    for (int C = 1; C < NG; ++C) y[C][i] *= alf;
    xc[i] = z0;
    y[0][i] = (float)z0;
    const float zi = fabsf(alf) * yinf[i];
    gam[i] = fmaxf((float)p.ga, 0.0f);
    if (rig) {
      // FP32 slope applied to the generators and to yinf (slope rounding +
      // product: 2u), FP64 center update, gamma rounded to FP32, evaluation
      // error of the parameters; rY and r are rounded up, so they bound the
      // exact sums
      const double ep = 2.0 * (double)kU * ((double)fabsf(alf) * (double)rY + (double)zi) + 2.0 * kU64 * fabs(z0) +
                        (double)kU * (double)gam[i] + (double)p.dg + (double)kEta;
      yinf[i] = round_up_f(((double)zi + ep) * (1.0 + 2.0 * kU64));
    } else {
      yinf[i] = zi;
    }
    rnext[i] = fabsf(alf) * r + gam[i];
  }

  int n_occ_new = n_occ;
  if (POL == SPK_AFFINE_FIXED) {
    // affine-fixed: every new term goes straight into the condensed coefficient
#pragma unroll
    for (int i = 0; i < 4; ++i) yinf[i] = rig ? round_up_f((double)yinf[i] + (double)gam[i]) : yinf[i] + gam[i];
  } else {
    // affine-truncate(k): candidates are the occupied old slots 1..n_occ
    // (magnitude = column L1 norm over the box's H rows) and the H new terms
    // (magnitude gamma_j); keep the k largest, ties to the lower candidate
    // index (old slots in slot order, then new terms by neuron index).
    constexpr int SEG = S::SEG;
    const int ch = lane % SEG;
    uint32_t kold[S::NS];
    kold[0] = 0u;
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const float mu = seg_allsum<SEG>((fabsf(y[C][0]) + fabsf(y[C][1])) + (fabsf(y[C][2]) + fabsf(y[C][3])));
      kold[C] = __float_as_uint(mu) & 0x7fffffffu;
    }
    uint32_t knew[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) knew[i] = __float_as_uint(gam[i]) & 0x7fffffffu;
    // old candidates this lane counts: slots C with (C-1) % SEG == ch
    constexpr int Q = (S::NS - 1 + SEG - 1) / SEG;
    uint32_t mine[Q];
    bool minev[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) { mine[q] = 0u; minev[q] = false; }
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const int q = (C - 1) / SEG;
      const bool sel = ((C - 1) % SEG) == ch;
      mine[q] = sel ? kold[C] : mine[q];
      minev[q] = sel ? (C <= n_occ) : minev[q];
    }
    // radix select of the k-th largest key, most significant bit first.  It
    // stops as soon as the keys >= T are exactly k (the remaining bits cannot
    // change the kept set), and does not start when at most k keys are
    // nonzero (T = 0 keeps them all).  The loop exits when every box of the
    // wave is done, so the ballots always run on the whole wave.
    uint32_t T = 0u;
    {
      int cpos = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) cpos += seg_count<SEG>(minev[q] && mine[q] != 0u, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) cpos += seg_count<SEG>(knew[i] != 0u, lane);
      bool done = cpos <= k;
#pragma unroll 1
      for (int bit = 30; bit >= 0; --bit) {
        if (__ballot(!done) == 0ull) break;
        const uint32_t Tc = T | (1u << bit);
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) cnt += seg_count<SEG>(minev[q] && mine[q] >= Tc, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) cnt += seg_count<SEG>(knew[i] >= Tc, lane);
        const bool take = !done && cnt >= k;
        T = take ? Tc : T;
        done = done || (take && cnt == k);
      }
    }
    const uint32_t tau = T;
    int cgt = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) cgt += seg_count<SEG>(minev[q] && mine[q] > tau, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) cgt += seg_count<SEG>(knew[i] > tau, lane);
    const int need = k - cgt;
    // old slots: equal-to-tau ones ranked by slot
    uint32_t eqm = 0u, keep_old = 0u;
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const bool v = C <= n_occ;
      eqm |= (v && kold[C] == tau) ? (1u << C) : 0u;
    }
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const bool v = C <= n_occ;
      const bool kp = v && (kold[C] > tau || (kold[C] == tau && __popc(eqm & ((1u << C) - 1u)) < need));
      keep_old |= kp ? (1u << C) : 0u;
    }
    const int n_eq_old = __popc(eqm);
    // new terms: rank among equal keys by neuron (row) index
    int run = n_eq_old;
#pragma unroll
    for (int i = 0; i < 4; ++i) run += seg_count_below<SEG>(knew[i] == tau, lane);
    bool keepnew[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool eq = knew[i] == tau;
      keepnew[i] = knew[i] > tau || (eq && run < need);
      run += eq ? 1 : 0;
    }
    // free slots (dropped old, then empty ones up to k) receive the kept new
    // terms in increasing slot order by increasing neuron index
    const uint32_t occm = (n_occ >= 31) ? 0xfffffffeu : ((1u << (n_occ + 1)) - 2u);
    const uint32_t kmsk = (k >= 31) ? 0xfffffffeu : ((1u << (k + 1)) - 2u);
    uint32_t freem = (occm & ~keep_old) | (kmsk & ~occm);
    if (S::BPW == 1) freem = __builtin_amdgcn_readfirstlane(freem);
    int rk = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) rk += seg_count_below<SEG>(keepnew[i], lane);
    int slot[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      slot[i] = keepnew[i] ? nth_set_bit(freem, rk) : -1;
      rk += keepnew[i] ? 1 : 0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double zi = (double)yinf[i];
#pragma unroll
      for (int C = 1; C < S::NS; ++C) {
        if ((freem >> C) & 1u) {
          zi += (double)fabsf(y[C][i]);
          y[C][i] = (slot[i] == C) ? gam[i] : 0.0f;
        }
      }
      zi += keepnew[i] ? 0.0 : (double)gam[i];
      // rigorous: FP64 sum of at most NS + 1 terms, rounded upwards
      yinf[i] = rig ? round_up_f(zi * (1.0 + (double)(S::NS + 3) * kU64)) : (float)zi;
    }
    if (sent != nullptr) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (slot[i] >= 4) {
          sent[slot[i]] = gam[i];
          ((int*)sent)[S::NS + slot[i]] = 4 * ch + i;
        }
      }
    }
    if (rec != nullptr) {
      if (ch == 0) {
        // a rolled loop: unrolled, its 32 per-slot constants would be hoisted
        // out of the box loop and held (spilled) for the whole kernel
#pragma unroll 1
        for (int C = 0; C < 32; ++C) {
          const bool fr = (freem >> C) & 1u;
          if (!fr) rec[C] = (C == 0 || C <= k) ? (int16_t)-1 : (int16_t)-2;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (slot[i] >= 0) rec[slot[i]] = (int16_t)(4 * ch + i);
    }
    n_occ_new = (n_occ + S::H < k) ? n_occ + S::H : k;
  }
  if (rig) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      yinf[i] = round_up_f((double)yinf[i] + ((double)cK * (double)rnext[i] + (double)cD * fabs(xc[i])) *
                                                 (1.0 + 1.52587890625e-05) + (double)kEta);
  }
  return n_occ_new;
}

// Reduce the VALU partial sums of output tile tp of box b over the four
// K-row groups of the wave and store them in the LDS vectors.
template <class S>
__device__ __forceinline__ void store_partials(LdsState<S>& sm, int b, int tp, int g, int c, float sx, double sd) {
  sx = rows_allsum(sx);
  sd = rows_allsum(sd);
  if (g == 0) {
    sm.vinf[b * S::H + 16 * tp + c] = sx;
    sm.vc[b * S::H + 16 * tp + c] = sd;
  }
}

// VALU work that rides along an MFMA pass: none (later column tiles) or the
// FP64 center and |W| xinf (VA_CENTER).
enum { VA_NONE = 0, VA_CENTER = 1 };

// Column tile n of the wave's single box (H = 256) through one H -> H layer.
// The A fragments stream from L2 in MFMA order (fragment (t, tp) is the
// q = t MT + tp th one); a ring of PF fragments keeps PF - 1 loads in flight
// so their latency hides behind the MFMAs, and the next K block's B fragment
// and vectors are read from LDS one block ahead.
template <class S, int VA>
__device__ __forceinline__ void single_box_pass(LdsState<S>& sm, const f4* Wl, int n, int lane) {
  constexpr int MT = S::MT, PF = 8;
  static_assert(S::BPW == 1 && MT % PF == 0, "one box per wave; the ring index repeats every K block");
  const int g = lane >> 4, c = lane & 15;
  f4 acc[MT];
  float px[MT];
  double pd[MT];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    acc[tp] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
    px[tp] = 0.0f;
    pd[tp] = 0.0;
  }
  const f4* Wq = Wl + lane;
  f4 ring[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) ring[p] = Wq[p * 64];
  f4 bn = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, g)];
  f4 xn = {0.0f, 0.0f, 0.0f, 0.0f};
  double dn[4] = {0.0, 0.0, 0.0, 0.0};
  if (VA != VA_NONE) {
    xn = *(const f4*)&sm.vinf[4 * g];
#pragma unroll
    for (int j = 0; j < 4; ++j) dn[j] = sm.vc[4 * g + j];
  }
#pragma unroll 1
  for (int t = 0; t < MT; ++t) {
    const f4 bfr = bn, vx = xn;
    double vd[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) vd[j] = dn[j];
    const int t1 = min(t + 1, MT - 1);
    bn = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 4 * t1 + g)];
    if (VA != VA_NONE) {
      xn = *(const f4*)&sm.vinf[16 * t1 + 4 * g];
#pragma unroll
      for (int j = 0; j < 4; ++j) dn[j] = sm.vc[16 * t1 + 4 * g + j];
    }
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      const f4 w = ring[tp % PF];
      const int qn = min(t * MT + tp + PF, MT * MT - 1);   // past the end: a harmless reload
      ring[tp % PF] = Wq[(size_t)qn * 64];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[tp] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[j], bfr[j], acc[tp], 0, 0, 0);
        if (VA != VA_NONE) {
          px[tp] = fmaf(fabsf(w[j]), vx[j], px[tp]);
          pd[tp] = fma((double)w[j], vd[j], pd[tp]);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    if (VA != VA_NONE) store_partials<S>(sm, 0, tp, g, c, px[tp], pd[tp]);
    *(f4*)&sm.tile[taddr<S>(0, 16 * n + c, 4 * tp + g)] = acc[tp];
  }
  __syncthreads();
}

// Both column tiles of the wave's single box (H = 256, 32 term slots) in one
// sweep over W: every A fragment feeds the MFMAs of both tiles, so W streams
// from L2 once per layer for the generators instead of once per tile.  The
// VALU products (FP64 center, |W| xinf, |W| u) run first in a sweep of their
// own and are stored before the MFMA sweep: their partial sums beside the two
// accumulator sets would not fit the register file (interleaved, the kernel
// spills inside the loop and runs 15 % slower).  Each accumulator sees the same
// product sequence as in single_box_pass, so the results are identical.
template <class S, int VA>
__device__ __forceinline__ void single_box_pass2(LdsState<S>& sm, const f4* Wl, int lane) {
  constexpr int MT = S::MT, PF = 8;
  static_assert(S::BPW == 1 && S::NT == 2 && MT % PF == 0, "one box per wave, two column tiles");
  const int g = lane >> 4, c = lane & 15;
  const f4* Wq = Wl + lane;
  if (VA != VA_NONE) {
    float px[MT];
    double pd[MT];
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      px[tp] = 0.0f;
      pd[tp] = 0.0;
    }
    f4 ring[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) ring[p] = Wq[p * 64];
#pragma unroll 1
    for (int t = 0; t < MT; ++t) {
      const f4 vx = *(const f4*)&sm.vinf[16 * t + 4 * g];
      double vd[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) vd[j] = sm.vc[16 * t + 4 * g + j];
#pragma unroll
      for (int tp = 0; tp < MT; ++tp) {
        const f4 w = ring[tp % PF];
        const int qn = min(t * MT + tp + PF, MT * MT - 1);
        ring[tp % PF] = Wq[(size_t)qn * 64];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          px[tp] = fmaf(fabsf(w[j]), vx[j], px[tp]);
          pd[tp] = fma((double)w[j], vd[j], pd[tp]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) store_partials<S>(sm, 0, tp, g, c, px[tp], pd[tp]);
  }
  f4 acc0[MT], acc1[MT];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    acc0[tp] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
    acc1[tp] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
  }
  f4 ring[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) ring[p] = Wq[p * 64];
  f4 bn0 = *(const f4*)&sm.tile[taddr<S>(0, c, g)];
  f4 bn1 = *(const f4*)&sm.tile[taddr<S>(0, 16 + c, g)];
#pragma unroll 1
  for (int t = 0; t < MT; ++t) {
    const f4 b0 = bn0, b1 = bn1;
    const int t1 = min(t + 1, MT - 1);
    bn0 = *(const f4*)&sm.tile[taddr<S>(0, c, 4 * t1 + g)];
    bn1 = *(const f4*)&sm.tile[taddr<S>(0, 16 + c, 4 * t1 + g)];
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      const f4 w = ring[tp % PF];
      const int qn = min(t * MT + tp + PF, MT * MT - 1);   // past the end: a harmless reload
      ring[tp % PF] = Wq[(size_t)qn * 64];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc0[tp] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[j], b0[j], acc0[tp], 0, 0, 0);
        acc1[tp] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[j], b1[j], acc1[tp], 0, 0, 0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    *(f4*)&sm.tile[taddr<S>(0, c, 4 * tp + g)] = acc0[tp];
    *(f4*)&sm.tile[taddr<S>(0, 16 + c, 4 * tp + g)] = acc1[tp];
  }
  __syncthreads();
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// Split 8 floats into BF16 hi and lo parts (round to nearest even each): the
// residual v - hi is exact in FP32.
__device__ __forceinline__ void split_bf16(const f4& a, const f4& b, bf8& hi, bf8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float v = i < 4 ? a[i] : b[i - 4];
    const __bf16 h = (__bf16)v;
    hi[i] = h;
    lo[i] = (__bf16)(v - (float)h);
  }
}

// Column tile n of the wave's single box (H = 256) with split-BF16 generator
// products: W_hi X_hi + W_hi X_lo + W_lo X_hi on the 16x16x32 BF16 MFMA, K in
// blocks of 32 rows (lane (g, c) holds rows 32 t2 + 8 g .. + 7 of column c).
// The FP64 center and the |W| products run first on VALU over the FP32
// fragments (first pass only).
template <class S, int VA>
__device__ __forceinline__ void single_box_pass_split(LdsState<S>& sm, const f4* Wl, const uint32_t* Wbl, int n,
                                                      int lane) {
  constexpr int MT = S::MT, MT2 = MT / 2, PF = 4;
  static_assert(S::BPW == 1 && MT % PF == 0, "one box per wave; the ring index repeats every K block");
  const int g = lane >> 4, c = lane & 15;
  f4 acc[MT];
  float px[MT];
  double pd[MT];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    acc[tp] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
    px[tp] = 0.0f;
    pd[tp] = 0.0;
  }
  if (VA != VA_NONE) {
    const f4* Wq = Wl + lane;
    f4 ring[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) ring[p] = Wq[p * 64];
#pragma unroll 1
    for (int t = 0; t < MT; ++t) {
      const f4 vx = *(const f4*)&sm.vinf[16 * t + 4 * g];
      double vd[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) vd[j] = sm.vc[16 * t + 4 * g + j];
#pragma unroll
      for (int tp = 0; tp < MT; ++tp) {
        const f4 w = ring[tp % PF];
        const int qn = min(t * MT + tp + PF, MT * MT - 1);
        ring[tp % PF] = Wq[(size_t)qn * 64];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          px[tp] = fmaf(fabsf(w[j]), vx[j], px[tp]);
          pd[tp] = fma((double)w[j], vd[j], pd[tp]);
        }
      }
    }
  }
  // fragment (t2, tp): two 16-byte vectors (8 hi, 8 lo BF16) per lane
  const u4v* Bq = (const u4v*)Wbl + 2 * lane;
  u4v rh[PF], rl[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    rh[p] = Bq[(size_t)p * 128];
    rl[p] = Bq[(size_t)p * 128 + 1];
  }
#pragma unroll 1
  for (int t2 = 0; t2 < MT2; ++t2) {
    const f4 b0 = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 8 * t2 + 2 * g)];
    const f4 b1 = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 8 * t2 + 2 * g + 1)];
    bf8 xh, xl;
    split_bf16(b0, b1, xh, xl);
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      const bf8 ah = __builtin_bit_cast(bf8, rh[tp % PF]);
      const bf8 al = __builtin_bit_cast(bf8, rl[tp % PF]);
      const int qn = min(t2 * MT + tp + PF, MT2 * MT - 1);   // past the end: a harmless reload
      rh[tp % PF] = Bq[(size_t)qn * 128];
      rl[tp % PF] = Bq[(size_t)qn * 128 + 1];
      acc[tp] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xh, acc[tp], 0, 0, 0);
      acc[tp] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xl, acc[tp], 0, 0, 0);
      acc[tp] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, xh, acc[tp], 0, 0, 0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    if (VA != VA_NONE) store_partials<S>(sm, 0, tp, g, c, px[tp], pd[tp]);
    *(f4*)&sm.tile[taddr<S>(0, 16 * n + c, 4 * tp + g)] = acc[tp];
  }
  __syncthreads();
}

typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// Split 8 scaled floats into FP16 hi and lo parts (round to nearest even
// each): hi = RNE16(v), lo = RNE16(v - hi); v - hi is exact in FP32.
__device__ __forceinline__ void split_f16(const f4& a, const f4& b, h8& hi, h8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float v = i < 4 ? a[i] : b[i - 4];
    const _Float16 h = (_Float16)v;
    hi[i] = h;
    lo[i] = (_Float16)(v - (float)h);
  }
}

// Column tile n of the wave's single box (H = 256) with scaled split-FP16
// generator products.  Each column c of X is scaled by a power of two 2^s_c
// that puts its max |x| in [2^14, 2^15) (FP16 range, no overflow); W' = W 2^sW
// is the layer's split copy with unscale factor wsc.  W'_hi X'_hi +
// W'_hi X'_lo + W'_lo X'_hi run on the 16x16x32 FP16 MFMA with FP32
// accumulation, and the result is unscaled by the two powers of two.  The
// FP64 center and the |W| products run first on VALU over the FP32 fragments
// (first pass only).  Returns the sum of 2^-s_c over the tile's nonzero
// generator columns (the same value on every lane), which scales the
// absolute part of the split error.
template <class S, int VA>
__device__ __forceinline__ float single_box_pass_f16(LdsState<S>& sm, const f4* Wl, const uint32_t* Whl, float wsc,
                                                     int n, int lane) {
  constexpr int MT = S::MT, MT2 = MT / 2, PF = 4;
  static_assert(S::BPW == 1 && MT % PF == 0, "one box per wave; the ring index repeats every K block");
  const int g = lane >> 4, c = lane & 15;
  if (VA != VA_NONE) {
    // VALU products first, reduced and stored before the MFMA loop so their
    // partial sums are not live beside the accumulators
    float px[MT];
    double pd[MT];
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      px[tp] = 0.0f;
      pd[tp] = 0.0;
    }
    const f4* Wq = Wl + lane;
    f4 ring[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) ring[p] = Wq[p * 64];
#pragma unroll 1
    for (int t = 0; t < MT; ++t) {
      const f4 vx = *(const f4*)&sm.vinf[16 * t + 4 * g];
      double vd[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) vd[j] = sm.vc[16 * t + 4 * g + j];
#pragma unroll
      for (int tp = 0; tp < MT; ++tp) {
        const f4 w = ring[tp % PF];
        const int qn = min(t * MT + tp + PF, MT * MT - 1);
        ring[tp % PF] = Wq[(size_t)qn * 64];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          px[tp] = fmaf(fabsf(w[j]), vx[j], px[tp]);
          pd[tp] = fma((double)w[j], vd[j], pd[tp]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) store_partials<S>(sm, 0, tp, g, c, px[tp], pd[tp]);
  }
  // this lane's column scale: lanes c, c + 16, c + 32, c + 48 hold the
  // column's rows 8 g .. 8 g + 7 of every 32-row block
  float m = 0.0f;
#pragma unroll 1
  for (int t2 = 0; t2 < MT2; ++t2) {
    const f4 b0 = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 8 * t2 + 2 * g)];
    const f4 b1 = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 8 * t2 + 2 * g + 1)];
#pragma unroll
    for (int j = 0; j < 4; ++j) m = fmaxf(m, fmaxf(fabsf(b0[j]), fabsf(b1[j])));
  }
  m = rows_allmax(m);
  const int ex = (int)((__float_as_uint(m) >> 23) & 0xffu) - 127;   // floor(log2 m); -127 for 0
  const int sh = min(14 - ex, 126);
  const float sc = __uint_as_float((uint32_t)(sh + 127) << 23);
  const float isc = __uint_as_float((uint32_t)(127 - sh) << 23);
  // sum of isc over the generator columns (column 0 of the first tile holds
  // the center, whose product is not used) with a nonzero entry
  float ssum = (m > 0.0f && (n > 0 || c > 0)) ? isc : 0.0f;
  ssum = seg_allsum<16>(ssum);
  f4 acc[MT];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) acc[tp] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
  // fragment (t2, tp): two 16-byte vectors (8 hi, 8 lo FP16) per lane
  const u4v* Bq = (const u4v*)Whl + 2 * lane;
  u4v rh[PF], rl[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    rh[p] = Bq[(size_t)p * 128];
    rl[p] = Bq[(size_t)p * 128 + 1];
  }
#pragma unroll 1
  for (int t2 = 0; t2 < MT2; ++t2) {
    const f4 b0 = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 8 * t2 + 2 * g)];
    const f4 b1 = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 8 * t2 + 2 * g + 1)];
    h8 xh, xl;
    split_f16(b0 * sc, b1 * sc, xh, xl);
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      const h8 ah = __builtin_bit_cast(h8, rh[tp % PF]);
      const h8 al = __builtin_bit_cast(h8, rl[tp % PF]);
      const int qn = min(t2 * MT + tp + PF, MT2 * MT - 1);   // past the end: a harmless reload
      rh[tp % PF] = Bq[(size_t)qn * 128];
      rl[tp % PF] = Bq[(size_t)qn * 128 + 1];
      acc[tp] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, xh, acc[tp], 0, 0, 0);
      acc[tp] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, xl, acc[tp], 0, 0, 0);
      acc[tp] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, xh, acc[tp], 0, 0, 0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) *(f4*)&sm.tile[taddr<S>(0, 16 * n + c, 4 * tp + g)] = (acc[tp] * wsc) * isc;
  __syncthreads();
  return ssum;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Column tile n of the wave's single box (H = 256) with FP64 generator
// products: the 16x16x4 FP64 MFMA in the same fragment order as the FP32 one
// (lane (g, c) feeds W[16t' + c][16t + 4g + j] and X[16t + 4g + j][16n + c],
// both widened exactly from FP32) with FP64 accumulation (the operands use
// the FP32 MFMA's lane layout, the accumulators another one, see below); the
// results are rounded to FP32 in the tile.  In tile 0 the lanes of column 0 feed the FP64
// center x0 from sm.vc instead of its FP32 copy, so the center W x0 comes out
// of the same MFMA in FP64 (column 0) and no VALU center sweep is needed;
// |W| xinf (VA_CENTER) runs on VALU beside it.
template <class S, int VA>
__device__ __forceinline__ void single_box_pass_f64(LdsState<S>& sm, const f4* Wl, int n, int lane) {
  constexpr int MT = S::MT, PF = 8;
  static_assert(S::BPW == 1 && MT % PF == 0, "one box per wave; the ring index repeats every K block");
  const int g = lane >> 4, c = lane & 15;
  const bool ctr = (n == 0) && (c == 0);
  d4 acc[MT];
  float px[MT];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    acc[tp] = (d4){0.0, 0.0, 0.0, 0.0};
    px[tp] = 0.0f;
  }
  const f4* Wq = Wl + lane;
  f4 ring[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) ring[p] = Wq[p * 64];
#pragma unroll 1
  for (int t = 0; t < MT; ++t) {
    const f4 bfr = *(const f4*)&sm.tile[taddr<S>(0, 16 * n + c, 4 * t + g)];
    double bd[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bd[j] = ctr ? sm.vc[16 * t + 4 * g + j] : (double)bfr[j];
    f4 vx = {0.0f, 0.0f, 0.0f, 0.0f};
    if (VA != VA_NONE) vx = *(const f4*)&sm.vinf[16 * t + 4 * g];
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      const f4 w = ring[tp % PF];
      const int qn = min(t * MT + tp + PF, MT * MT - 1);   // past the end: a harmless reload
      ring[tp % PF] = Wq[(size_t)qn * 64];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[tp] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)w[j], bd[j], acc[tp], 0, 0, 0);
        if (VA != VA_NONE) px[tp] = fmaf(fabsf(w[j]), vx[j], px[tp]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
    if (VA != VA_NONE) {
      const float sx = rows_allsum(px[tp]);
      if (g == 0) sm.vinf[16 * tp + c] = sx;
    }
    // the FP64 MFMA's accumulator layout differs from the FP32 one (measured):
    // lane (g, c) holds rows 16 tp + g + 4 i (i = 0..3) of column c
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (ctr) sm.vc[16 * tp + g + 4 * i] = acc[tp][i];
      sm.tile[taddr<S>(0, 16 * n + c, 4 * tp + i) + g] = (float)acc[tp][i];
    }
  }
  __syncthreads();
}

// Column tile n of every box of the wave (H < 256: several boxes) through one
// H -> H layer.  This K block's A fragments are held for every output tile
// (MT is small here) and reused box after box.
template <class S, int VA>
__device__ __forceinline__ void multi_box_pass(LdsState<S>& sm, const f4* Wl, int n, int lane) {
  constexpr int H = S::H, MT = S::MT, BPW = S::BPW;
  const int g = lane >> 4, c = lane & 15;
  f4 acc[MT][BPW];
  float px[MT][BPW];
  double pd[MT][BPW];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      acc[tp][b] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
      px[tp][b] = 0.0f;
      pd[tp][b] = 0.0;
    }
  }
  // the next K block's A fragments load while this one's MFMAs run
  f4 wn[MT];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) wn[tp] = Wl[(size_t)tp * 64 + lane];
#pragma unroll 1
  for (int t = 0; t < MT; ++t) {
    f4 w[MT];
    const f4* Wt = Wl + (size_t)min(t + 1, MT - 1) * MT * 64 + lane;
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      w[tp] = wn[tp];
      wn[tp] = Wt[tp * 64];
    }
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      const f4 bfr = *(const f4*)&sm.tile[taddr<S>(b, 16 * n + c, 4 * t + g)];
      f4 vx = {0.0f, 0.0f, 0.0f, 0.0f};
      double vd[4] = {0.0, 0.0, 0.0, 0.0};
      if (VA != VA_NONE) {
        vx = *(const f4*)&sm.vinf[b * H + 16 * t + 4 * g];
#pragma unroll
        for (int j = 0; j < 4; ++j) vd[j] = sm.vc[b * H + 16 * t + 4 * g + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int tp = 0; tp < MT; ++tp) {
          acc[tp][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[tp][j], bfr[j], acc[tp][b], 0, 0, 0);
          if (VA != VA_NONE) {
            px[tp][b] = fmaf(fabsf(w[tp][j]), vx[j], px[tp][b]);
            pd[tp][b] = fma((double)w[tp][j], vd[j], pd[tp][b]);
          }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) {
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      if (VA != VA_NONE) store_partials<S>(sm, b, tp, g, c, px[tp][b], pd[tp][b]);
      *(f4*)&sm.tile[taddr<S>(b, 16 * n + c, 4 * tp + g)] = acc[tp][b];
    }
  }
  __syncthreads();
}

// One hidden layer (index a among the H -> H layers) from owner layout to
// owner layout through the LDS tile.  Ends with the pre-activation form of
// the next activation: centers with bias (FP64), generators, condensed term,
// error radius; passengers receive the bias too.
template <class S, int NPASS, int PREC = SPK_PREC_F32>
__device__ __forceinline__ void hidden_layer(const NetDev& net, LdsState<S>& sm, int a, double (&xc)[4],
                                             f4 (&y)[S::NS], float (&yinf)[4], float (&e)[4],
                                             const float (&u)[4], int lane, bool rigorous) {
  constexpr int H = S::H, NT = S::NT, NS = S::NS, BPW = S::BPW, SEG = S::SEG;
  const int bo = lane / SEG;
  const int ch = lane % SEG;
  const float cK = net.cK;

  // ---- owner layout -> LDS ----
#pragma unroll
  for (int C = 0; C < NS; ++C) {
    const f4 v = y[C];
    *(f4*)&sm.tile[taddr<S>(bo, C, ch)] = v;
  }
  {
    f4 v1 = {yinf[0], yinf[1], yinf[2], yinf[3]};
    *(f4*)&sm.vinf[4 * lane] = v1;
#pragma unroll
    for (int i = 0; i < 4; ++i) sm.vc[4 * lane + i] = xc[i];
  }
  __syncthreads();

  // ---- generators on MFMA, center in FP64, |W| xinf on VALU ----
  const f4* Wl = (const f4*)net.Wp + (size_t)a * (H * H / 4);
  float sc_sum = 0.0f;   // split-FP16: sum of the column unscale factors
  if constexpr (PREC == SPK_PREC_F16X3) {
    static_assert(BPW == 1, "scaled split-FP16 products are built for one box per wave");
    const uint32_t* Whl = net.Wh + (size_t)a * (H * H);   // H*H (hi, lo) pairs of 16-bit values
    const float wsc = net.wsh[a];
    sc_sum = single_box_pass_f16<S, VA_CENTER>(sm, Wl, Whl, wsc, 0, lane);
#pragma unroll 1
    for (int n = 1; n < NT; ++n) sc_sum += single_box_pass_f16<S, VA_NONE>(sm, Wl, Whl, wsc, n, lane);
    sc_sum *= 1.0f + 3.814697265625e-06f;   // 1 + 2^-18: FP32 sums of at most 32 powers of two
  } else if constexpr (PREC == SPK_PREC_BF16X3) {
    static_assert(BPW == 1, "split-BF16 products are built for one box per wave");
    const uint32_t* Wbl = net.Wb + (size_t)a * (H * H);   // H*H (hi, lo) pairs of 16-bit values
    single_box_pass_split<S, VA_CENTER>(sm, Wl, Wbl, 0, lane);
#pragma unroll 1
    for (int n = 1; n < NT; ++n) single_box_pass_split<S, VA_NONE>(sm, Wl, Wbl, n, lane);
  } else if constexpr (PREC == SPK_PREC_F64) {
    static_assert(BPW == 1, "FP64 products are built for one box per wave");
    single_box_pass_f64<S, VA_CENTER>(sm, Wl, 0, lane);
#pragma unroll 1
    for (int n = 1; n < NT; ++n) single_box_pass_f64<S, VA_NONE>(sm, Wl, n, lane);
  } else if constexpr (BPW == 1 && NT == 2) {
    single_box_pass2<S, VA_CENTER>(sm, Wl, lane);
  } else if constexpr (BPW == 1) {
    single_box_pass<S, VA_CENTER>(sm, Wl, 0, lane);
#pragma unroll 1
    for (int n = 1; n < NT; ++n) single_box_pass<S, VA_NONE>(sm, Wl, n, lane);
  } else {
    multi_box_pass<S, VA_CENTER>(sm, Wl, 0, lane);
#pragma unroll 1
    for (int n = 1; n < NT; ++n) multi_box_pass<S, VA_NONE>(sm, Wl, n, lane);
  }
  __syncthreads();
#pragma unroll
  for (int C = 1; C < NS; ++C) {
    const f4 v = *(const f4*)&sm.tile[taddr<S>(bo, C, ch)];
    y[C] = v;
  }
  {
    const f4 xi = *(const f4*)&sm.vinf[4 * lane];
    const f4 bh = *(const f4*)&net.bh[(size_t)a * H + 4 * ch];
    const f4 eb = *(const f4*)&net.ebh[(size_t)a * H + 4 * ch];
    const double grow = 1.0 + 2.0 * (double)cK;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xc[i] = sm.vc[4 * lane + i] + (double)bh[i];
      y[0][i] = (float)xc[i];
#pragma unroll
      for (int C = NS - NPASS; C < NS; ++C) y[C][i] += bh[i];
      // rigorous: the FP32 sum |W| xinf is within cK of exact; the input yinf
      // already holds this layer's a-priori product rounding; e takes the
      // bias addition (and the split-FP16 absolute terms below)
      yinf[i] = rigorous ? round_up_f((double)xi[i] * grow) : xi[i];
      e[i] = eb[i] + (float)(2.0 * kU64) * (float)fabs(xc[i]);
      // absolute split-FP16 errors, per column c with scale 2^s_c: FP16
      // underflow of X entries (<= 2^-13 scaled, times |W_hi + W_lo| <=
      // 2 |W|) and W residuals too small for a normal lo part (D_j times
      // max |x'| < 2^15); dwt_j bounds 2^-12 sum_k |W_jk| + D_j 2^(15 - sW)
      if constexpr (PREC == SPK_PREC_F16X3) e[i] = fmaf(net.dwt[(size_t)a * H + 4 * ch + i], sc_sum, e[i]) * kGrow;
      (void)u;
    }
  }
  __syncthreads();
}

// LDS scratch of the first hidden layer inside the (then unused) tile: per
// box the three dense columns [3][H], after them per box the single-entry
// table written by the first activation (NS values, then NS row indices).
template <class S>
__device__ __forceinline__ float* first_layer_dense(LdsState<S>& sm, int bo) {
  return sm.tile + bo * (3 * S::H);
}
template <class S>
__device__ __forceinline__ float* first_layer_sent(LdsState<S>& sm, int bo) {
  static_assert(S::BPW * (3 * S::H + 2 * S::NS) <= S::TILE, "first-layer scratch must fit the tile");
  return sm.tile + S::BPW * (3 * S::H) + bo * (2 * S::NS);
}

// The first H -> H layer (Table 2 matrix multiplication) in owner layout,
// without the matrix core.  Entering it, the generator slots hold the s <= 3
// input-axis columns (slots 1..3, dense: kept old terms keep their slots) and,
// in slots 4..klast, new terms of the first truncation (Section 3.3), each a
// single entry gamma_j on row j.  The center and the dense columns are
// multiplied by W in FP64 and rounded once: at this layer the FP32 rounding of
// the input-axis columns is what the chord slopes of narrow straddling neurons
// amplify most in the later layers.  A single-entry column is the scaled
// weight column W[:, j] gamma_j (one FP32 rounding, the value any FP32
// summation order gives).  |W| xinf runs in FP32.  Lane ch owns rows 4ch..4ch+3 of its box and streams W from the
// 4x4-blocked copy (one coalesced 64-byte row block per lane and k block); the
// box's vectors are LDS broadcasts.  In the rigorous mode the input yinf
// already holds the a-priori rounding of this layer for the constant cK, which
// covers this evaluation too.
template <class S, bool RIG>
__device__ __forceinline__ void first_hidden_layer(const NetDev& net, LdsState<S>& sm, double (&xc)[4],
                                                   f4 (&y)[S::NS], float (&yinf)[4], float (&e)[4],
                                                   const float (&u)[4], int lane, int klast) {
  constexpr int H = S::H, NS = S::NS, SEG = S::SEG;
  const int bo = lane / SEG;
  const int ch = lane % SEG;
  float* dense = first_layer_dense<S>(sm, bo);
  const float* sent = first_layer_sent<S>(sm, bo);
  // ---- owner layout -> LDS (the box's vectors and dense columns) ----
#pragma unroll
  for (int c = 0; c < 3; ++c) *(f4*)&dense[c * H + 4 * ch] = y[c + 1];
  {
    f4 v1 = {yinf[0], yinf[1], yinf[2], yinf[3]};
    *(f4*)&sm.vinf[4 * lane] = v1;
#pragma unroll
    for (int i = 0; i < 4; ++i) sm.vc[4 * lane + i] = xc[i];
  }
  __syncthreads();
  const double* vc = sm.vc + bo * H;
  const float* vi = sm.vinf + bo * H;
  const f4* Wr = (const f4*)net.Wr + 4 * ch;   // hidden layer 0
  double a0[4], a1[4], a2[4], a3[4];
  float px[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a0[i] = 0.0; a1[i] = 0.0; a2[i] = 0.0; a3[i] = 0.0;
    px[i] = 0.0f;
  }
  // one k block (4 columns of W, rows 4ch..4ch+3) of the products
  auto block = [&](int kb, const f4 (&w)[4]) {
    const f4 d1 = *(const f4*)&dense[4 * kb];
    const f4 d2 = *(const f4*)&dense[H + 4 * kb];
    const f4 d3 = *(const f4*)&dense[2 * H + 4 * kb];
    const f4 xi = *(const f4*)&vi[4 * kb];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double x0 = vc[4 * kb + j];
      const double x1 = (double)d1[j], x2 = (double)d2[j], x3 = (double)d3[j];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double wd = (double)w[i][j];
        a0[i] = fma(wd, x0, a0[i]);
        a1[i] = fma(wd, x1, a1[i]);
        a2[i] = fma(wd, x2, a2[i]);
        a3[i] = fma(wd, x3, a3[i]);
        px[i] = fmaf(fabsf(w[i][j]), xi[j], px[i]);
      }
    }
  };
  // four k blocks per step: their 16 weight loads are in flight together
  static_assert((H / 4) % 4 == 0, "k blocks in fours");
#pragma unroll 1
  for (int kb = 0; kb < H / 4; kb += 4) {
    f4 w[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) w[b][i] = Wr[(size_t)(kb + b) * H + i];
#pragma unroll
    for (int b = 0; b < 4; ++b) block(kb + b, w[b]);
  }
  // ---- single-entry columns: y[C] = W[:, j] gamma_j; slots past klast are
  // empty (assigned here so that no slot stays live across the loop above).
  // With one box per wave the products go through the slots' own (free) LDS
  // rows, four slots per step, so that the step's 16 weight loads are in
  // flight together; slots past klast load row 0 and store zeros.
  if constexpr (S::BPW == 1) {
    static_assert((NS - 4) % 4 == 0, "slots in fours");
    static_assert(3 * H + 2 * NS <= 4 * H, "the dense columns and the table lie below slot 4");
#pragma unroll 1
    for (int C0 = 4; C0 < NS; C0 += 4) {
      f4 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int C = C0 + q;
        const bool on = C <= klast;
        const float g = sent[C];
        const int j = on ? ((const int*)sent)[NS + C] : 0;
        const float* wc = net.Wr + ((size_t)(j >> 2) * H + 4 * ch) * 4 + (j & 3);
        // the load is used unconditionally (a select of it becomes a branch
        // around it); the FMA with +0 turns the zero product into +0
        const float gs = on ? g : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[q][i] = fmaf(wc[4 * i], gs, 0.0f);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) *(f4*)&sm.tile[taddr<S>(0, C0 + q, ch)] = v[q];
    }
#pragma unroll
    for (int C = 4; C < NS; ++C) y[C] = *(const f4*)&sm.tile[taddr<S>(0, C, ch)];
  } else {
#pragma unroll
    for (int C = 4; C < NS; ++C) {
      f4 v = {0.0f, 0.0f, 0.0f, 0.0f};
      if (C <= klast) {
        const float g = sent[C];
        const int j = ((const int*)sent)[NS + C];
        const float* wc = net.Wr + ((size_t)(j >> 2) * H + 4 * ch) * 4 + (j & 3);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = wc[4 * i] * g;
      }
      y[C] = v;
    }
  }
  __syncthreads();
  const f4 bh = *(const f4*)&net.bh[4 * ch];
  const f4 eb = *(const f4*)&net.ebh[4 * ch];
  const double grow = 1.0 + 2.0 * (double)net.cK;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    xc[i] = a0[i] + (double)bh[i];
    y[0][i] = (float)xc[i];
    y[1][i] = (float)a1[i];
    y[2][i] = (float)a2[i];
    y[3][i] = (float)a3[i];
    yinf[i] = RIG ? round_up_f((double)px[i] * grow) : px[i];
    e[i] = eb[i] + (float)(2.0 * kU64) * (float)fabs(xc[i]);
  }
  (void)u;
}

struct OutVals {
  double y0;    // center
  float r;      // radius (rounded up in the rigorous mode)
  float err;    // rigorous mode: rounding of the output layer itself
};

// Output layer (H -> 1) and range read-off, reduced over the box's segment
// (every lane of the segment gets the same values).  pass[] receives the
// passengers' plain evaluations f(x).  In the rigorous mode the input yinf
// already holds the a-priori rounding of these products (cK, cD); err adds
// the rounding of |w| yinf, of the radius sum, of the output bias and of the
// center.
template <class S, int NPASS>
__device__ __forceinline__ OutVals output_layer(const NetDev& net, const double (&xc)[4], const f4 (&y)[S::NS],
                                                const float (&yinf)[4], const float (&u)[4], int lane,
                                                float (&pass)[NPASS > 0 ? NPASS : 1], bool rig = false) {
  constexpr int NS = S::NS, SEG = S::SEG, NG = NS - NPASS;
  const int ch = lane % SEG;
  const float cK = net.cK;
  (void)u;
  const f4 wv = *(const f4*)&net.wL[4 * ch];
  double p0 = 0.0;
  float pinf = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    p0 = fma((double)wv[i], xc[i], p0);
    pinf = fmaf(fabsf(wv[i]), yinf[i], pinf);
  }
  p0 = seg_allsum_d<SEG>(p0);
  pinf = seg_allsum<SEG>(pinf);
  double rd = 0.0;
#pragma unroll
  for (int C = 1; C < NG; ++C) {
    float pc = wv[0] * y[C][0];
    pc = fmaf(wv[1], y[C][1], pc);
    pc = fmaf(wv[2], y[C][2], pc);
    pc = fmaf(wv[3], y[C][3], pc);
    rd += (double)fabsf(seg_allsum<SEG>(pc));
  }
  rd += (double)pinf;
#pragma unroll
  for (int C = NG; C < NS; ++C) {
    float pc = wv[0] * y[C][0];
    pc = fmaf(wv[1], y[C][1], pc);
    pc = fmaf(wv[2], y[C][2], pc);
    pc = fmaf(wv[3], y[C][3], pc);
    pass[C - NG] = seg_allsum<SEG>(pc) + net.bL;
  }
  OutVals o;
  o.y0 = p0 + (double)net.bL;
  if (rig) {
    const double rr = rd * (1.0 + (double)(NS + 2) * kU64);
    o.r = round_up_f(rr);
    o.err = round_up_f((2.0 * (double)cK * (double)pinf + (double)net.eL + 4.0 * kU64 * fabs(o.y0)) *
                           (1.0 + 4.0 * kU64) + (double)kEta);
  } else {
    o.r = (float)rd;
    o.err = 0.0f;
  }
  return o;
}

// FP32 enclosure [lo, hi] of center +- (radius + w) with outward rounding.
// w is the rigorous rounding radius err (rigorous = true) or the
// floating-point tolerance margin 2^-18 (|center| + radius).  Non-finite
// results become [-inf, +inf].
__device__ __forceinline__ double tolerance_margin(const OutVals& o) {
  return 3.814697265625e-06 * (fabs(o.y0) + (double)o.r) + 1e-30;
}

__device__ __forceinline__ void enclose(const OutVals& o, bool rigorous, float& lo, float& hi) {
  const double margin = rigorous ? (double)o.err : tolerance_margin(o);
  const double s = ((double)o.r + margin) * (1.0 + 4.0 * kU64);
  lo = round_down_f(o.y0 - s);
  hi = round_up_f(o.y0 + s);
  if (!(lo <= hi) || !(lo > -INFINITY) || !(hi < INFINITY)) {
    lo = -INFINITY;
    hi = INFINITY;
  }
}

// Layer 0 applied to an affine input with FP64 center cc, FP32 axes ax[q]
// (q < 3; unused axes zero) and per-coordinate input error radius ein, plus
// NPASS passenger points.  Owner layout: rows 4ch..4ch+3.
template <class S, int NPASS>
__device__ __forceinline__ void layer0_affine(const NetDev& net, int ch, const double (&cc)[3],
                                              const float (&ax)[3][3], const float (&ein)[3],
                                              const float (&pts)[NPASS > 0 ? NPASS : 1][3], double (&xc)[4],
                                              f4 (&y)[S::NS], float (&yinf)[4], float (&e)[4]) {
  constexpr int NG = S::NS - NPASS;
  const f4* W0 = (const f4*)net.W0;   // rows padded to 4 floats
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = 4 * ch + i;
    const f4 w = W0[R];
    const float bb = net.b0[R];
    xc[i] = fma((double)w.z, cc[2], fma((double)w.y, cc[1], fma((double)w.x, cc[0], (double)bb)));
    const float cmag = (float)(fabs((double)w.x * cc[0]) + fabs((double)w.y * cc[1]) + fabs((double)w.z * cc[2])) +
                       fabsf(bb);
    y[0][i] = (float)xc[i];
    // generator columns 1..3 = W0 times the box axes; the rest start empty
    const float g0 = fmaf(w.z, ax[0][2], fmaf(w.y, ax[0][1], w.x * ax[0][0]));
    const float g1 = fmaf(w.z, ax[1][2], fmaf(w.y, ax[1][1], w.x * ax[1][0]));
    const float g2 = fmaf(w.z, ax[2][2], fmaf(w.y, ax[2][1], w.x * ax[2][0]));
    const float gmag = fabsf(w.x) * (fabsf(ax[0][0]) + fabsf(ax[1][0]) + fabsf(ax[2][0])) +
                       fabsf(w.y) * (fabsf(ax[0][1]) + fabsf(ax[1][1]) + fabsf(ax[2][1])) +
                       fabsf(w.z) * (fabsf(ax[0][2]) + fabsf(ax[1][2]) + fabsf(ax[2][2]));
    y[1][i] = g0;
    y[2][i] = g1;
    y[3][i] = g2;
#pragma unroll
    for (int C = 4; C < NG; ++C) y[C][i] = 0.0f;
#pragma unroll
    for (int C = NG; C < S::NS; ++C) {
      const int q = C - NG;
      y[C][i] = fmaf(w.z, pts[q][2], fmaf(w.y, pts[q][1], fmaf(w.x, pts[q][0], bb)));
    }
    yinf[i] = 0.0f;
    e[i] = (net.c3 * gmag + (float)(8.0 * kU64) * cmag + fabsf(w.x) * ein[0] + fabsf(w.y) * ein[1] +
            fabsf(w.z) * ein[2]) * kGrow + kEta;
  }
}

}  // namespace spk
