// Batched range bound of an MLP over boxes (Procedure 1) on gfx950.
//
// Per wavefront and group of BPW boxes (see affine_core.h / affine_stack.h):
//   layer 0 (3 -> H)      VALU, owner layout (box -> affine form, Procedure 1
//                         step 1; Table 2 matrix multiplication)
//   activation + condense owner layout (eq. affine_func_update, Table 3,
//                         Section 3.3 fixed / truncate)
//   hidden layers         MFMA 16x16x4 FP32 for the generator columns Y = W X;
//                         the center column W x0 in FP64 and the products
//                         |W| xinf and |W| u (rounding-error column) on VALU
//   output layer (H -> 1) range read-off (eq. def_range) and classification
//                         (Procedure 1).
//
// The center runs in FP64 because it carries the cancellation of every
// layer: in FP32 its rounding grows to ~1e-4 of the bound on 8-layer
// networks, while the generators and the condensed term stay accurate.
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

template <class S, int ACT, int POL>
__global__ __launch_bounds__(64, 1) void bound_kernel(NetDev net, BoundJob job) {
  __shared__ __attribute__((aligned(16))) LdsState<S> sm;
  constexpr int NS = S::NS, BPW = S::BPW, SEG = S::SEG;
  const int lane = threadIdx.x;
  const int bo = lane / SEG;
  const int ch = lane % SEG;
  const int64_t ngroups = (job.n + BPW - 1) / BPW;
  const int L = net.L;

  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t box = grp * BPW + bo;
    const bool valid = box < job.n;
    double cc[3];
    float ax[3][3], ein[3], pts[1][3] = {{0.0f, 0.0f, 0.0f}};
    box_input(job, box, valid, cc, ax, ein);
    double xc[4];
    f4 y[NS];
    float yinf[4], e[4], u[4];
    layer0_affine<S, 0>(net, ch, cc, ax, ein, pts, xc, y, yinf, e);
    int n_occ = job.s;
    for (int a = 0; a < L - 1; ++a) {
      int16_t* rec = nullptr;
      if (job.slot_src != nullptr && valid) rec = job.slot_src + ((size_t)a * job.n + box) * 32;
      n_occ = activate<S, ACT, POL, 0>(xc, y, yinf, e, u, n_occ, job.k, net.cK, net.cD, net.omega0, lane, rec);
      if (a == L - 2) break;
      hidden_layer<S, 0>(net, sm, a, xc, y, yinf, e, u, lane, job.rigorous != 0);
    }
    float pass[1];
    const OutVals o = output_layer<S, 0>(net, xc, y, yinf, u, lane, pass);
    if (valid && ch == 0) {
      float lo, hi;
      enclose(o, job.rigorous != 0, lo, hi);
      if (job.lo) job.lo[box] = lo;
      if (job.hi) job.hi[box] = hi;
      if (job.label) job.label[box] = (lo > 0.0f) ? (uint8_t)SPK_POSITIVE
                                      : (hi < 0.0f) ? (uint8_t)SPK_NEGATIVE : (uint8_t)SPK_UNKNOWN;
      if (job.center) job.center[box] = (float)o.y0;
      if (job.radius) job.radius[box] = o.r;
      if (job.err) job.err[box] = job.rigorous ? o.err : round_up_f(tolerance_margin(o));
    }
  }
}

template <class S, int ACT, int POL>
static hipError_t launch_one(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  const int64_t ngroups = (job.n + S::BPW - 1) / S::BPW;
  int64_t blocks = (int64_t)num_cus * 4;
  if (blocks > ngroups) blocks = ngroups;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((bound_kernel<S, ACT, POL>), dim3((unsigned)blocks), dim3(64), 0, stream, net, job);
  return hipGetLastError();
}

template <int H, int NT, int POL>
static hipError_t launch_act(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  switch (net.act) {
    case SPK_ACT_RELU: return launch_one<Shape<H, NT>, SPK_ACT_RELU, POL>(net, job, stream, num_cus);
    case SPK_ACT_ELU: return launch_one<Shape<H, NT>, SPK_ACT_ELU, POL>(net, job, stream, num_cus);
    case SPK_ACT_SIN: return launch_one<Shape<H, NT>, SPK_ACT_SIN, POL>(net, job, stream, num_cus);
  }
  return hipErrorInvalidValue;
}

template <int H>
static hipError_t launch_h(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  if (job.policy == SPK_AFFINE_FIXED) return launch_act<H, 1, SPK_AFFINE_FIXED>(net, job, stream, num_cus);
  if (job.k <= 15) return launch_act<H, 1, SPK_AFFINE_TRUNCATE>(net, job, stream, num_cus);
  return launch_act<H, 2, SPK_AFFINE_TRUNCATE>(net, job, stream, num_cus);
}

spk_status launch_bound(const spk_net* net, const BoundJob& job, hipStream_t stream, int num_cus) {
  if (job.n <= 0) return SPK_OK;
  hipError_t err;
  switch (net->dev.H) {
    case 32: err = launch_h<32>(net->dev, job, stream, num_cus); break;
    case 64: err = launch_h<64>(net->dev, job, stream, num_cus); break;
    case 128: err = launch_h<128>(net->dev, job, stream, num_cus); break;
    case 256: err = launch_h<256>(net->dev, job, stream, num_cus); break;
    default: return SPK_E_UNSUPPORTED;
  }
  return err == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
