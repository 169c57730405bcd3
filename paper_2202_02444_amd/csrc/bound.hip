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
#include "bound_group.h"

namespace spk {

// Each workgroup takes one contiguous range of box groups, so that the boxes
// it reads and the lo / hi / label entries it writes share cache lines with
// its own neighbours only (interleaved groups would spread every output line
// over several XCDs' L2s and write it back piecemeal).  With one box per
// wave, the results of each run of 64 boxes are collected in LDS and stored
// with one coalesced write per array, instead of a 4-byte write per box that
// the L2 would write back as a partial line again and again while the wave
// works on the next boxes.
template <class S, int ACT, int POL, int PREC>
__global__ __launch_bounds__(64, 1) void bound_kernel(NetDev net, BoundJob job) {
  __shared__ __attribute__((aligned(16))) LdsState<S> sm;
  __shared__ BoxResult stash[64];
  const int lane = (int)threadIdx.x;
  const int64_t ngroups = (job.n + S::BPW - 1) / S::BPW;
  const int64_t g0 = ngroups * blockIdx.x / gridDim.x, g1 = ngroups * (blockIdx.x + 1) / gridDim.x;
  if constexpr (S::BPW == 1) {
    for (int64_t base = g0; base < g1; base += 64) {
      const int cnt = (int)min((int64_t)64, g1 - base);
#pragma unroll 1
      for (int j = 0; j < cnt; ++j) {
        BoxResult r;
        bound_group<S, ACT, POL, PREC>(net, job, sm, base + j, lane, &r);
        if (lane == 0) stash[j] = r;
      }
      __syncthreads();
      if (lane < cnt) {
        const BoxResult r = stash[lane];
        const int64_t box = base + lane;
        if (job.lo) job.lo[box] = r.lo;
        if (job.hi) job.hi[box] = r.hi;
        if (job.label) job.label[box] = r.label;
        if (job.center) job.center[box] = r.center;
        if (job.radius) job.radius[box] = r.radius;
        if (job.err) job.err[box] = r.err;
      }
      __syncthreads();
    }
  } else {
    for (int64_t grp = g0; grp < g1; ++grp) bound_group<S, ACT, POL, PREC>(net, job, sm, grp, lane);
  }
}

template <class S, int ACT, int POL, int PREC>
static hipError_t launch_one(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  const int64_t ngroups = (job.n + S::BPW - 1) / S::BPW;
  int64_t blocks = (int64_t)num_cus * 4;
  if (blocks > ngroups) blocks = ngroups;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((bound_kernel<S, ACT, POL, PREC>), dim3((unsigned)blocks), dim3(64), 0, stream, net, job);
  return hipGetLastError();
}

template <int H, int NT, int POL, int PREC>
static hipError_t launch_act(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  switch (net.act) {
    case SPK_ACT_RELU: return launch_one<Shape<H, NT>, SPK_ACT_RELU, POL, PREC>(net, job, stream, num_cus);
    case SPK_ACT_ELU: return launch_one<Shape<H, NT>, SPK_ACT_ELU, POL, PREC>(net, job, stream, num_cus);
    case SPK_ACT_SIN: return launch_one<Shape<H, NT>, SPK_ACT_SIN, POL, PREC>(net, job, stream, num_cus);
  }
  return hipErrorInvalidValue;
}

template <int H, int PREC>
static hipError_t launch_h(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  if (job.policy == SPK_AFFINE_FIXED) return launch_act<H, 1, SPK_AFFINE_FIXED, PREC>(net, job, stream, num_cus);
  if (job.k <= 15) return launch_act<H, 1, SPK_AFFINE_TRUNCATE, PREC>(net, job, stream, num_cus);
  return launch_act<H, 2, SPK_AFFINE_TRUNCATE, PREC>(net, job, stream, num_cus);
}

spk_status launch_bound(const spk_net* net, const BoundJob& job, hipStream_t stream, int num_cus) {
  if (job.policy == SPK_AFFINE_FULL) return launch_full(net, job, stream, num_cus);
  if (job.n <= 0) return SPK_OK;
  hipError_t err;
  if (job.prec == SPK_PREC_BF16X3 || job.prec == SPK_PREC_F16X3 || job.prec == SPK_PREC_F64) {
    // split and FP64 products are built for one box per wave (hidden width 256)
    if (net->dev.H != 256) return SPK_E_UNSUPPORTED;
    if (job.prec == SPK_PREC_BF16X3)
      err = launch_h<256, SPK_PREC_BF16X3>(net->dev, job, stream, num_cus);
    else if (job.prec == SPK_PREC_F16X3)
      err = launch_h<256, SPK_PREC_F16X3>(net->dev, job, stream, num_cus);
    else
      err = launch_h<256, SPK_PREC_F64>(net->dev, job, stream, num_cus);
    return err == hipSuccess ? SPK_OK : SPK_E_DEVICE;
  }
  switch (net->dev.H) {
    case 32: err = launch_h<32, SPK_PREC_F32>(net->dev, job, stream, num_cus); break;
    case 64: err = launch_h<64, SPK_PREC_F32>(net->dev, job, stream, num_cus); break;
    case 128: err = launch_h<128, SPK_PREC_F32>(net->dev, job, stream, num_cus); break;
    case 256: err = launch_h<256, SPK_PREC_F32>(net->dev, job, stream, num_cus); break;
    default: return SPK_E_UNSUPPORTED;
  }
  return err == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
