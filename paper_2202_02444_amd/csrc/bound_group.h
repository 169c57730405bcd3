// One group of BPW boxes of a bound job through the whole network
// (Procedure 1), shared by the single-network and the batched kernels.
#pragma once

#include "affine_stack.h"

namespace spk {

// Box of the bound job as an affine input: FP64 center, FP32 axes and the
// input error radius that covers the rounding of the axes.
__device__ __forceinline__ void box_input(const BoundJob& job, int64_t box, bool valid, double (&cc)[3],
                                          float (&ax)[3][3], float (&ein)[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    cc[d] = 0.0;
    ein[d] = 0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) ax[q][d] = 0.0f;
  }
  if (!valid) return;
  if (job.mode == IN_GENERAL) {
#pragma unroll
    for (int d = 0; d < 3; ++d) cc[d] = (double)job.a[3 * box + d];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int d = 0; d < 3; ++d) ax[q][d] = (q < job.s) ? job.b[(box * job.s + q) * 3 + d] : 0.0f;
    return;
  }
  float lo[3], hi[3];
  if (job.mode == IN_AABB) {
#pragma unroll
    for (int d = 0; d < 3; ++d) { lo[d] = job.a[3 * box + d]; hi[d] = job.b[3 * box + d]; }
  } else {
    cell_box(job.cells[box], job.level, job.dom_lo, job.dom_hi, lo, hi);
  }
  // center and half-width of the FP32 box, exactly, in FP64 (Procedure 3:
  // x_c = (x_l + x_u)/2, v = x_u - x_c); the half-width is then rounded to
  // FP32 for the generator, its rounding kept in ein
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    cc[d] = 0.5 * ((double)lo[d] + (double)hi[d]);
    const double h = (double)hi[d] - cc[d];
    ax[d][d] = (float)h;
    ein[d] = 2.0f * kU * fabsf((float)h) + kEta;
  }
}

// Results of one box (identical in every lane of its segment).
struct BoxResult {
  float lo, hi, center, radius, err;
  uint8_t label;
};

// With `out` null the box results are written to the job's arrays by the
// segment's first lane; otherwise (one box per wave) they are returned in
// *out on every lane and the caller writes them.
template <class S, int ACT, int POL, int PREC = SPK_PREC_F32>
__device__ __forceinline__ void bound_group(const NetDev& net, const BoundJob& job, LdsState<S>& sm, int64_t grp,
                                            int lane, BoxResult* out = nullptr) {
  constexpr int NS = S::NS, BPW = S::BPW, SEG = S::SEG;
  const int bo = lane / SEG;
  const int ch = lane % SEG;
  const int L = net.L;
  const int64_t box = grp * BPW + bo;
  const bool valid = box < job.n;
  double cc[3];
  float ax[3][3], ein[3], pts[1][3] = {{0.0f, 0.0f, 0.0f}};
  box_input(job, box, valid, cc, ax, ein);
  if (job.nonfinite != nullptr && valid && ch == 0) {
    // device status: boxes whose input coordinates are not all finite
    bool fin = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      fin = fin && isfinite(cc[d]);
#pragma unroll
      for (int q = 0; q < 3; ++q) fin = fin && isfinite(ax[q][d]);
    }
    if (!fin) atomicAdd(job.nonfinite, 1ull);
  }
  double xc[4];
  f4 y[NS];
  float yinf[4], e[4], u[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  layer0_affine<S, 0>(net, ch, cc, ax, ein, pts, xc, y, yinf, e);
  int n_occ = job.s;
  const bool rig = job.rigorous != 0;
  // the next layer's generator products: FP32 or split-BF16 rounding bound
  // (FP64 products: the FP64 accumulation bound, and the FP32 rounding of
  // each stored generator, relative to the stored value, folded by activate)
  const float cKg = PREC == SPK_PREC_BF16X3 ? net.cKs
                    : (PREC == SPK_PREC_F16X3 ? net.cKh : (PREC == SPK_PREC_F64 ? net.cD : net.cK));
  const float uY = PREC == SPK_PREC_F64 ? kU * kGrow : 0.0f;
  if constexpr (S::BPW == 1) {
    {
      // first activation; with a hidden H -> H layer after it, that layer's
      // generator columns are the input axes and single entries: row-owner
      // products, the dense ones in FP64
      int16_t* rec = (job.slot_src != nullptr && valid) ? job.slot_src + (size_t)box * 32 : nullptr;
      float* sent = POL == SPK_AFFINE_TRUNCATE ? first_layer_sent<S>(sm, bo) : nullptr;
      n_occ = activate<S, ACT, POL, 0>(xc, y, yinf, e, u, n_occ, job.k, cKg, net.cD, net.omega0, lane, rec, sent,
                                       rig, 0.0f);
    }
    if (L > 2) {
      const int klast = POL == SPK_AFFINE_TRUNCATE ? job.k : 3;
      if (job.rigorous)
        first_hidden_layer<S, true>(net, sm, xc, y, yinf, e, u, lane, klast);
      else
        first_hidden_layer<S, false>(net, sm, xc, y, yinf, e, u, lane, klast);
      for (int a = 1; a < L - 1; ++a) {
        int16_t* rec = nullptr;
        if (job.slot_src != nullptr && valid) rec = job.slot_src + ((size_t)a * job.n + box) * 32;
        n_occ = activate<S, ACT, POL, 0>(xc, y, yinf, e, u, n_occ, job.k, cKg, net.cD, net.omega0, lane, rec,
                                         nullptr, rig, uY);
        if (a == L - 2) break;
        hidden_layer<S, 0, PREC>(net, sm, a, xc, y, yinf, e, u, lane, job.rigorous != 0);
      }
    }
  } else {
    // several boxes per wave (H < 256): every hidden layer on the MFMA
    for (int a = 0; a < L - 1; ++a) {
      int16_t* rec = nullptr;
      if (job.slot_src != nullptr && valid) rec = job.slot_src + ((size_t)a * job.n + box) * 32;
      n_occ = activate<S, ACT, POL, 0>(xc, y, yinf, e, u, n_occ, job.k, cKg, net.cD, net.omega0, lane, rec,
                                       nullptr, rig);
      if (a == L - 2) break;
      hidden_layer<S, 0, PREC>(net, sm, a, xc, y, yinf, e, u, lane, job.rigorous != 0);
    }
  }
  float pass[1];
  const OutVals o = output_layer<S, 0>(net, xc, y, yinf, u, lane, pass, rig);
  BoxResult r;
  enclose(o, job.rigorous != 0, r.lo, r.hi);
  // band r >= 0 (surface sampling, Section 4.6): POSITIVE means f > r on the
  // box, NEGATIVE f < -r (r = 0: Procedure 1)
  r.label = (r.lo > job.band) ? (uint8_t)SPK_POSITIVE : (r.hi < -job.band) ? (uint8_t)SPK_NEGATIVE
                                                                            : (uint8_t)SPK_UNKNOWN;
  r.center = (float)o.y0;
  r.radius = o.r;
  r.err = job.rigorous ? o.err : round_up_f(tolerance_margin(o));
  if (out != nullptr) {
    *out = r;
  } else if (valid && ch == 0) {
    if (job.lo) job.lo[box] = r.lo;
    if (job.hi) job.hi[box] = r.hi;
    if (job.label) job.label[box] = r.label;
    if (job.center) job.center[box] = r.center;
    if (job.radius) job.radius[box] = r.radius;
    if (job.err) job.err[box] = r.err;
  }
}

}  // namespace spk
