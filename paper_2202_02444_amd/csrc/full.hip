// Range bound with the affine-full policy (Section 3.3: no condensation; every
// nonlinearity adds one new term per neuron and all of them are kept) on
// gfx950, for hidden width 128 or 256, one box per wavefront (at width 128
// lanes 32..63 own no rows and only join the matrix-core sweep).
//
// The generator matrix of a box grows by H columns per hidden layer (3 input
// axes, then one diagonal block per activation), to 32 + (L - 2) H columns,
// too large for registers or LDS: it lives in a per-wave slice of a device
// workspace, column-major (column c = rows 0..H-1, contiguous), so that a
// row-owner lane (rows 4 ch .. 4 ch + 3) reads or writes 16 bytes of a column
// and the 64 lanes cover it in one coalesced kilobyte.
//
// Columns 0..31 form tile 0: the input-axis generators in columns 1..3 (the
// other columns zero); the diagonal block of activation a (a = 0 .. L - 3)
// occupies columns 32 + 256 a .. 32 + 256 a + 255.  The stored values are the
// generators before the next activation's slope: the slope alpha_k of row k
// multiplies row k of every stored column when the next layer reads it.
//
// Hidden layer a (W = W_a, the layer's H x H weights) turns the stored matrix
// Y and the previous activation's (alpha, beta, gamma) into the next one:
//   old columns:      Y <- W diag(alpha) Y, in place, 32 columns at a time
//                     (rows scaled while staged into the LDS tile, products
//                     on the FP32 matrix core, the same sweep as the
//                     truncated policy's two-tile pass), with the row sums of
//                     |Y| for the next range;
//   new block:        column j = W[:, j] gamma_j, written from the 4x4-blocked
//                     copy of W by the row owners, with their row sums;
//   center:           W x' + b in FP64 in the same row-owner sweep.
// The activation (Table 3) then works on the rows: range radius = row sum of
// |Y| (plus, in the rounding-bounded mode, the error radius e), and the
// output layer reads every stored column once more: the radius is
// sum_c |w . (alpha o Y)[:, c]| + sum_j |w_j| gamma_j.
//
// Rounding-bounded mode (the default): every rounding is bounded a priori and
// put into the new term of its neuron, which is a fresh symbol like gamma_j
// (two fresh symbols of one neuron merge into one with the summed radius):
//   * the exact pre-activation lies within e_j of the computed form, where e
//     bounds the generator products (cK |W| (|alpha| rY)), the products of the
//     diagonal block (u |W| gamma), the FP64 center and the bias; the
//     linearisation is taken on the range widened by e;
//   * gamma'_j = gamma_j + |alpha_j| e_j + the rounding of alpha Y, of the
//     FP64 center update, of gamma itself and the parameters' evaluation
//     error.
// The paper's arithmetic ignores rounding (Section 3.4) and encloses the
// result with the floating-point tolerance margin.
#include "bound_group.h"

namespace spk {

namespace {

// One box per wave at hidden width HW: HW/16 row tiles, two 16-column tiles
// of generators, rows 4ch..4ch+3 owned by lane ch < HW/4.
template <int HW>
struct FShape {
  static constexpr int H = HW;
  static constexpr int MT = HW / 16;
  static constexpr int NT = 2;
  static constexpr int NS = 32;
  static constexpr int BPW = 1;
  static constexpr int SEG = HW / 4;
  static constexpr int TILE = NS * HW;
  static constexpr int SWM = ((HW / 4) < 16 ? (HW / 4) : 16) - 1;
};

template <int HW>
struct FullLds {
  LdsState<FShape<HW>> st;   // B tile of 32 columns, and the vectors x' (vc), v (vinf)
  float gam[HW];             // new-term radii gamma' of the last activation
};

// Table 3 activation of the four rows of this lane.  In: x (FP64 pre-activation
// center with bias), rY (row sum of |Y|, rounded up in the rounding-bounded
// mode), e (error radius; zero in the paper's arithmetic).  Out: the slope
// applied to the stored generators (alpha omega0 for the sine), the new-term
// radius g, the center x' and, rounding-bounded, the vector v whose product
// |W| v bounds the next layer's rounding.
template <int ACT>
__device__ __forceinline__ void act_full(double (&x)[4], const double (&rY)[4], const double (&e)[4], float omega0,
                                         bool rig, float cK, float cD, float (&al)[4], float (&g)[4],
                                         float (&v)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double x0 = x[i], ry = rY[i], ee = e[i];
    if (ACT == SPK_ACT_SIN) {
      // Table 2 constant multiplication by omega0 before sin (FP64)
      const double w = (double)omega0;
      x0 *= w;
      ry *= w;
      ee = ee * w + (rig ? 2.0 * kU64 * (fabs(x0) + ry) : 0.0);
    }
    double r = ry + ee;
    if (rig) r = r * (1.0 + 4.0 * kU64) + (double)kEta;
    const ActOut p = act_params<ACT>(x0 - r, x0 + r, x0);
    // slope on the stored generators (FP32), new center, new-term radius
    const double slope = ACT == SPK_ACT_SIN ? p.al * (double)omega0 : p.al;
    al[i] = (float)slope;
    const double z0 = fma(p.al, x0, p.be);
    x[i] = z0;
    const double ga = fmax(p.ga, 0.0);
    if (rig) {
      // |alpha| e, rounding of alpha Y (the FP32 slope and its product: 3u
      // relative on |alpha| rY), of the FP64 center update, of gamma itself
      // and the parameters' evaluation error
      const double aa = fabs(p.al);
      const double gt = ga + aa * ee + 3.0 * (double)kU * fabs(slope) * rY[i] * (1.0 + 4.0 * kU64) +
                        2.0 * kU64 * fabs(z0) + (double)kU * ga + (double)p.dg + (double)kEta;
      g[i] = round_up_f(gt * (1.0 + 8.0 * kU64));
      // the next layer's products: FP32 generators against W (cK on the
      // post-activation rows, |alpha| rY + gamma'), the diagonal block (u
      // gamma'), the FP64 center (cD |x'|)
      const double R = fabs((double)al[i]) * rY[i] * (1.0 + 2.0 * kU64) + (double)g[i];
      v[i] = round_up_f(((double)cK * R + (double)kU * (double)g[i] + (double)cD * fabs(z0)) * (1.0 + 8.0 * kU64) +
                        (double)kEta);
    } else {
      g[i] = (float)ga;
      v[i] = 0.0f;
    }
  }
}

template <int kH, int ACT>
__global__ __launch_bounds__(64, 1) void full_kernel(NetDev net, BoundJob job, float* ws, int64_t ncap) {
  using FS = FShape<kH>;
  __shared__ __attribute__((aligned(16))) FullLds<kH> sm;
  const int lane = (int)threadIdx.x;
  const int ch = lane;
  const bool own = ch < kH / 4;   // lane owns rows 4ch..4ch+3
  const int L = net.L;
  const bool rig = job.rigorous != 0;
  float* Yw = ws + (size_t)blockIdx.x * (size_t)kH * (size_t)ncap;   // this wave's generator matrix
  const int64_t b0 = job.n * blockIdx.x / gridDim.x, b1 = job.n * (blockIdx.x + 1) / gridDim.x;
#pragma unroll 1
  for (int64_t box = b0; box < b1; ++box) {
    double cc[3];
    float ax[3][3], ein[3], pts[1][3] = {{0.0f, 0.0f, 0.0f}};
    box_input(job, box, true, cc, ax, ein);
    if (job.nonfinite != nullptr && ch == 0) {
      bool fin = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        fin = fin && isfinite(cc[d]);
#pragma unroll
        for (int q = 0; q < 3; ++q) fin = fin && isfinite(ax[q][d]);
      }
      if (!fin) atomicAdd(job.nonfinite, 1ull);
    }
    // ---- layer 0 (3 -> H): center, axis generators, input error ----
    double x[4], rY[4], e[4];
    float al[4], g[4], v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = rY[i] = e[i] = 0.0;
    if (own) {
      double xc[4];
      f4 y[16];
      float yinf[4], e0[4];
      layer0_affine<Shape<256, 1>, 0>(net, ch, cc, ax, ein, pts, xc, y, yinf, e0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x[i] = xc[i];
        rY[i] = (double)fabsf(y[1][i]) + (double)fabsf(y[2][i]) + (double)fabsf(y[3][i]);
        if (rig) rY[i] *= 1.0 + 4.0 * kU64;
        e[i] = rig ? (double)e0[i] : 0.0;
      }
      // tile 0: columns 1..3 the axis generators, the rest zero
#pragma unroll
      for (int C = 0; C < 32; ++C) {
        f4 val = (C >= 1 && C <= 3) ? y[C] : (f4){0.0f, 0.0f, 0.0f, 0.0f};
        *(f4*)&Yw[(size_t)C * kH + 4 * ch] = val;
      }
    }
    act_full<ACT>(x, rY, e, net.omega0, rig, net.cK, net.cD, al, g, v);
    if (!own) {
      // lanes without rows carry zeros
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x[i] = rY[i] = 0.0;
        al[i] = g[i] = v[i] = 0.0f;
      }
    }
    int64_t ncols = 32;
    // ---- hidden layers ----
#pragma unroll 1
    for (int a = 0; a < L - 2; ++a) {
      // the previous activation's center, rounding vector and new-term radii
      // for every lane
      if (own) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          sm.st.vc[4 * ch + i] = x[i];
          sm.st.vinf[4 * ch + i] = v[i];
          sm.gam[4 * ch + i] = g[i];
        }
      }
      __syncthreads();
      // row-owner sweep over W (4x4 blocks): FP64 center, |W| v, and the new
      // block's columns W[:, j] gamma_j with their row sums
      const f4* Wr = (const f4*)net.Wr + (size_t)a * (kH * kH / 4) + 4 * ch;
      float* Yn = Yw + (size_t)ncols * kH + 4 * ch;
      double c0[4], rn[4];
      float pe[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c0[i] = 0.0;
        rn[i] = 0.0;
        pe[i] = 0.0f;
      }
#pragma unroll 1
      for (int kb = 0; kb < (own ? kH / 4 : 0); kb += 2) {
        f4 w[2][4];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) w[b][i] = Wr[(size_t)(kb + b) * kH + i];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int k0 = 4 * (kb + b);
          const f4 gj = *(const f4*)&sm.gam[k0];
          const f4 vj = *(const f4*)&sm.st.vinf[k0];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double xj = sm.st.vc[k0 + j];
            f4 col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float wij = w[b][i][j];
              c0[i] = fma((double)wij, xj, c0[i]);
              pe[i] = fmaf(fabsf(wij), vj[j], pe[i]);
              col[i] = wij * gj[j];
              rn[i] += (double)fabsf(col[i]);
            }
            *(f4*)&Yn[(size_t)(k0 + j) * kH] = col;
          }
        }
      }
      // old columns: Y <- W diag(alpha) Y, 32 at a time, in place
      double rs[4] = {0.0, 0.0, 0.0, 0.0};
      const f4* Wl = (const f4*)net.Wp + (size_t)a * (kH * kH / 4);
#pragma unroll 1
      for (int64_t c0t = 0; c0t < ncols; c0t += 32) {
        float* T = Yw + (size_t)c0t * kH + 4 * ch;
        __syncthreads();
        // eight columns' loads in flight per step
#pragma unroll 1
        for (int C0 = 0; C0 < (own ? 32 : 0); C0 += 8) {
          f4 buf[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) buf[q] = __builtin_nontemporal_load((const f4*)&T[(size_t)(C0 + q) * kH]);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            f4 val = buf[q];
#pragma unroll
            for (int i = 0; i < 4; ++i) val[i] *= al[i];
            *(f4*)&sm.st.tile[taddr<FS>(0, C0 + q, ch)] = val;
          }
        }
        __syncthreads();
        single_box_pass2<FS, VA_NONE>(sm.st, Wl, lane);
        if (own) {
#pragma unroll
          for (int C = 0; C < 32; ++C) {
            const f4 val = *(const f4*)&sm.st.tile[taddr<FS>(0, C, ch)];
#pragma unroll
            for (int i = 0; i < 4; ++i) rs[i] += (double)fabsf(val[i]);
            *(f4*)&T[(size_t)C * kH] = val;
          }
        }
      }
      ncols += kH;
      // pre-activation rows of the next activation
      const f4 f0 = {0.0f, 0.0f, 0.0f, 0.0f};
      const f4 bh = own ? *(const f4*)&net.bh[(size_t)a * kH + 4 * ch] : f0;
      const f4 eb = own ? *(const f4*)&net.ebh[(size_t)a * kH + 4 * ch] : f0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x[i] = c0[i] + (double)bh[i];
        rY[i] = rs[i] + rn[i];
        if (rig) {
          // FP64 sums of at most ncols + 1 terms
          rY[i] *= 1.0 + (double)(ncols + 4) * kU64;
          e[i] = ((double)pe[i] * (1.0 + 2.0 * (double)net.cK) + (double)eb[i] + 2.0 * kU64 * fabs(x[i])) *
                     (1.0 + 4.0 * kU64) + (double)kEta;
        } else {
          e[i] = 0.0;
        }
      }
      act_full<ACT>(x, rY, e, net.omega0, rig, net.cK, net.cD, al, g, v);
      if (!own) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x[i] = rY[i] = 0.0;
          al[i] = g[i] = v[i] = 0.0f;
        }
      }
    }
    // ---- output layer: center, sum over the stored columns of |w . alpha Y|,
    // and the last activation's new terms ----
    const f4 wv = own ? *(const f4*)&net.wL[4 * ch] : (f4){0.0f, 0.0f, 0.0f, 0.0f};
    float wa[4];
    double y0 = 0.0, rg = 0.0, perr = 0.0, cabs = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      wa[i] = wv[i] * al[i];
      y0 = fma((double)wv[i], x[i], y0);
      cabs += fabs((double)wv[i] * x[i]);
      rg += (double)fabsf(wv[i]) * (double)g[i];
      perr += (double)fabsf(wa[i]) * rY[i];
    }
    y0 = seg_allsum_d<64>(y0) + (double)net.bL;
    cabs = seg_allsum_d<64>(cabs);
    rg = seg_allsum_d<64>(rg);
    perr = seg_allsum_d<64>(perr);
    double rd = 0.0;
#pragma unroll 1
    for (int64_t c0t = 0; c0t < ncols; c0t += 32) {
      const float* T = Yw + (size_t)c0t * kH + 4 * ch;
      float p[32];
#pragma unroll
      for (int C = 0; C < 32; ++C) p[C] = 0.0f;
#pragma unroll 1
      for (int C0 = 0; C0 < (own ? 32 : 0); C0 += 8) {
        f4 buf[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) buf[q] = __builtin_nontemporal_load((const f4*)&T[(size_t)(C0 + q) * kH]);
#pragma unroll
        for (int q = 0; q < 8; ++q)
          p[C0 + q] = fmaf(wa[3], buf[q][3], fmaf(wa[2], buf[q][2], fmaf(wa[1], buf[q][1], wa[0] * buf[q][0])));
      }
#pragma unroll
      for (int C = 0; C < 32; ++C) rd += (double)fabsf(seg_allsum<64>(p[C]));
    }
    rd += rg;
    OutVals o;
    o.y0 = y0;
    if (rig) {
      // FP64 sums: ncols column terms, and the H-term sum of |w| gamma'
      o.r = round_up_f(rd * (1.0 + (double)(ncols + kH + 8) * kU64));
      // the dot products (cK on sum |w alpha Y|, plus the rounding of w
      // alpha), the FP64 center (an H-term dot product and the bias), the
      // output bias
      o.err = round_up_f(((double)(net.cK + 2.0f * kU) * perr * (1.0 + 2.0 * (double)net.cK) +
                          (double)net.cD * cabs * (1.0 + 4.0 * kU64) + (double)net.eL + 4.0 * kU64 * fabs(y0)) *
                             (1.0 + 8.0 * kU64) + (double)kEta);
    } else {
      o.r = (float)rd;
      o.err = 0.0f;
    }
    BoxResult r;
    enclose(o, rig, r.lo, r.hi);
    r.label = (r.lo > job.band) ? (uint8_t)SPK_POSITIVE : (r.hi < -job.band) ? (uint8_t)SPK_NEGATIVE
                                                                              : (uint8_t)SPK_UNKNOWN;
    r.center = (float)o.y0;
    r.radius = o.r;
    r.err = rig ? o.err : round_up_f(tolerance_margin(o));
    if (ch == 0) {
      if (job.lo) job.lo[box] = r.lo;
      if (job.hi) job.hi[box] = r.hi;
      if (job.label) job.label[box] = r.label;
      if (job.center) job.center[box] = r.center;
      if (job.radius) job.radius[box] = r.radius;
      if (job.err) job.err[box] = r.err;
    }
    __syncthreads();
  }
}

}  // namespace

// Columns of one box's generator matrix under affine-full.
static int64_t full_columns(int L, int H) { return 32 + (int64_t)(L - 2) * H; }

template <int HW>
static void launch_full_h(const NetDev& d, const BoundJob& job, float* ws, int64_t ncap, int64_t blocks,
                          hipStream_t stream) {
  switch (d.act) {
    case SPK_ACT_RELU:
      hipLaunchKernelGGL((full_kernel<HW, SPK_ACT_RELU>), dim3((unsigned)blocks), dim3(64), 0, stream, d, job, ws, ncap);
      break;
    case SPK_ACT_ELU:
      hipLaunchKernelGGL((full_kernel<HW, SPK_ACT_ELU>), dim3((unsigned)blocks), dim3(64), 0, stream, d, job, ws, ncap);
      break;
    default:
      hipLaunchKernelGGL((full_kernel<HW, SPK_ACT_SIN>), dim3((unsigned)blocks), dim3(64), 0, stream, d, job, ws, ncap);
      break;
  }
}

spk_status launch_full(const spk_net* net, const BoundJob& job, hipStream_t stream, int num_cus) {
  const NetDev& d = net->dev;
  if ((d.H != 256 && d.H != 128) || job.prec != SPK_PREC_F32) return SPK_E_UNSUPPORTED;
  if (job.n <= 0) return SPK_OK;
  int64_t blocks = (int64_t)num_cus * 4;
  if (blocks > job.n) blocks = job.n;
  if (blocks < 1) blocks = 1;
  const int64_t ncap = full_columns(d.L, d.H);
  const size_t bytes = (size_t)blocks * (size_t)d.H * (size_t)ncap * sizeof(float);
  float* ws = nullptr;
  if (hipMallocAsync((void**)&ws, bytes, stream) != hipSuccess) {
    (void)hipGetLastError();
    return SPK_E_NOMEM;
  }
  if (d.H == 256)
    launch_full_h<256>(d, job, ws, ncap, blocks, stream);
  else
    launch_full_h<128>(d, job, ws, ncap, blocks, stream);
  const hipError_t err = hipGetLastError();
  (void)hipFreeAsync(ws, stream);   // ordered after the launch on the stream
  return err == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
