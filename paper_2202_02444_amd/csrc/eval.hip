// Plain point evaluation f(x) of the MLP (the scalar evaluation that ray
// casting's convergence test and tests use).  Points are GEMM columns: the
// 16x16x4 MFMA accumulator layout of one layer is exactly the B-operand
// layout of the next, so activations stay in registers between layers.
#include "affine_stack.h"

namespace spk {

template <int ACT>
__device__ __forceinline__ float act_exact(float x, float omega0) {
  if (ACT == SPK_ACT_RELU) return fmaxf(x, 0.0f);
  if (ACT == SPK_ACT_ELU) return x > 0.0f ? x : expm1f(x);
  return sinf(omega0 * x);
}

template <int H, int ACT>
__global__ __launch_bounds__(64) void eval_kernel(NetDev net, int64_t n, const float* __restrict__ x,
                                                  float* __restrict__ f) {
  constexpr int MT = H / 16;
  // 16-point column tiles per pass: activations and accumulators take
  // 8 MT NTP = 128 registers (twice that spilled)
  constexpr int NTP = 256 / H;
  constexpr int PPP = 16 * NTP;       // points per pass
  const int lane = threadIdx.x;
  const int g = lane >> 4, c = lane & 15;
  const int64_t npass = (n + PPP - 1) / PPP;
  const int L = net.L;
  const f4* W0 = (const f4*)net.W0;
  for (int64_t pass = blockIdx.x; pass < npass; pass += gridDim.x) {
    f4 in[MT][NTP];
#pragma unroll
    for (int nn = 0; nn < NTP; ++nn) {
      const int64_t p = pass * PPP + 16 * nn + c;
      float px = 0.0f, py = 0.0f, pz = 0.0f;
      if (p < n) { px = x[3 * p]; py = x[3 * p + 1]; pz = x[3 * p + 2]; }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = 16 * t + 4 * g + j;
          const f4 w = W0[row];
          in[t][nn][j] = act_exact<ACT>(fmaf(w.z, pz, fmaf(w.y, py, fmaf(w.x, px, net.b0[row]))), net.omega0);
        }
      }
    }
    for (int a = 0; a < L - 2; ++a) {
      const f4* Wl = (const f4*)net.Wp + (size_t)a * (H * H / 4);
      f4 acc[MT][NTP];
#pragma unroll
      for (int tp = 0; tp < MT; ++tp) {
        const f4 bv = *(const f4*)&net.bh[(size_t)a * H + 16 * tp + 4 * g];
#pragma unroll
        for (int nn = 0; nn < NTP; ++nn) acc[tp][nn] = bv;
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
#pragma unroll
        for (int tp = 0; tp < MT; ++tp) {
          const f4 w = Wl[((size_t)t * MT + tp) * 64 + lane];
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int nn = 0; nn < NTP; ++nn)
              acc[tp][nn] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[j], in[t][nn][j], acc[tp][nn], 0, 0, 0);
        }
      }
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int nn = 0; nn < NTP; ++nn)
#pragma unroll
          for (int j = 0; j < 4; ++j) in[t][nn][j] = act_exact<ACT>(acc[t][nn][j], net.omega0);
    }
    // output layer: f = wL . h + bL, rows split over the four lane groups
#pragma unroll
    for (int nn = 0; nn < NTP; ++nn) {
      float s = 0.0f;
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const f4 w = *(const f4*)&net.wL[16 * t + 4 * g];
#pragma unroll
        for (int j = 0; j < 4; ++j) s = fmaf(w[j], in[t][nn][j], s);
      }
      s = rows_allsum(s);
      const int64_t p = pass * PPP + 16 * nn + c;
      if (g == 0 && p < n) f[p] = s + net.bL;
    }
  }
}

// Width 256: thirty-two points per pass, one column each of the bound
// kernel's LDS tile, through the same two-tile MFMA sweep (every weight
// fragment feeds both 16-point tiles; a ring of loads runs ahead).  Holding
// all 32 points' activations and accumulators in registers instead does not
// fit the register file.  Bias and activation are applied in row-owner layout
// (lane ch owns rows 4ch..4ch+3) between the layers; the output layer reduces
// each point's 256 products across the wave.
template <int ACT>
__global__ __launch_bounds__(64, 1) void eval256_kernel(NetDev net, int64_t n, const float* __restrict__ x,
                                                        float* __restrict__ f) {
  using S = Shape<256, 2>;
  __shared__ __attribute__((aligned(16))) LdsState<S> sm;
  const int lane = threadIdx.x;
  const int ch = lane;
  const int L = net.L;
  const int64_t npass = (n + 31) / 32;
  const f4* W0 = (const f4*)net.W0;
  f4 w0[4];
  float b0[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    w0[i] = W0[4 * ch + i];
    b0[i] = net.b0[4 * ch + i];
  }
  const f4 wv = *(const f4*)&net.wL[4 * ch];
  for (int64_t pass = blockIdx.x; pass < npass; pass += gridDim.x) {
    const int64_t p0 = pass * 32;
    // the pass's point coordinates (zeros past n) for every lane
    __syncthreads();
    if (lane < 32) {
      const int64_t p = p0 + lane;
#pragma unroll
      for (int d = 0; d < 3; ++d) sm.vinf[3 * lane + d] = p < n ? x[3 * p + d] : 0.0f;
    }
    __syncthreads();
    // layer 0 (3 -> 256)
#pragma unroll
    for (int C = 0; C < 32; ++C) {
      const float px = sm.vinf[3 * C], py = sm.vinf[3 * C + 1], pz = sm.vinf[3 * C + 2];
      f4 v;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        v[i] = act_exact<ACT>(fmaf(w0[i].z, pz, fmaf(w0[i].y, py, fmaf(w0[i].x, px, b0[i]))), net.omega0);
      *(f4*)&sm.tile[taddr<S>(0, C, ch)] = v;
    }
    __syncthreads();
    // hidden layers: products on the matrix core, then bias and activation
    for (int a = 0; a < L - 2; ++a) {
      single_box_pass2<S, VA_NONE>(sm, (const f4*)net.Wp + (size_t)a * (256 * 256 / 4), lane);
      const f4 bh = *(const f4*)&net.bh[(size_t)a * 256 + 4 * ch];
#pragma unroll
      for (int C = 0; C < 32; ++C) {
        f4 v = *(const f4*)&sm.tile[taddr<S>(0, C, ch)];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = act_exact<ACT>(v[i] + bh[i], net.omega0);
        *(f4*)&sm.tile[taddr<S>(0, C, ch)] = v;
      }
      __syncthreads();
    }
    // output layer: f = wL . h + bL; lane C keeps point C's value
    float mine = 0.0f;
#pragma unroll
    for (int C = 0; C < 32; ++C) {
      const f4 v = *(const f4*)&sm.tile[taddr<S>(0, C, ch)];
      const float s = seg_allsum<64>(fmaf(wv[3], v[3], fmaf(wv[2], v[2], fmaf(wv[1], v[1], wv[0] * v[0]))));
      mine = lane == C ? s : mine;
    }
    if (lane < 32 && p0 + lane < n) f[p0 + lane] = mine + net.bL;
  }
}

template <int H>
static hipError_t launch_eval_h(const NetDev& net, int64_t n, const float* x, float* f, hipStream_t stream,
                                int num_cus) {
  if constexpr (H == 256) {
    const int64_t npass = (n + 31) / 32;
    int64_t blocks = (int64_t)num_cus * 4;
    if (blocks > npass) blocks = npass;
    if (blocks < 1) blocks = 1;
    switch (net.act) {
      case SPK_ACT_RELU:
        hipLaunchKernelGGL(eval256_kernel<SPK_ACT_RELU>, dim3((unsigned)blocks), dim3(64), 0, stream, net, n, x, f);
        break;
      case SPK_ACT_ELU:
        hipLaunchKernelGGL(eval256_kernel<SPK_ACT_ELU>, dim3((unsigned)blocks), dim3(64), 0, stream, net, n, x, f);
        break;
      default:
        hipLaunchKernelGGL(eval256_kernel<SPK_ACT_SIN>, dim3((unsigned)blocks), dim3(64), 0, stream, net, n, x, f);
        break;
    }
    return hipGetLastError();
  } else {
    constexpr int PPP = 16 * (256 / H);
    const int64_t npass = (n + PPP - 1) / PPP;
    int64_t blocks = (int64_t)num_cus * 8;
    if (blocks > npass) blocks = npass;
    switch (net.act) {
      case SPK_ACT_RELU:
        hipLaunchKernelGGL((eval_kernel<H, SPK_ACT_RELU>), dim3((unsigned)blocks), dim3(64), 0, stream, net, n, x, f);
        break;
      case SPK_ACT_ELU:
        hipLaunchKernelGGL((eval_kernel<H, SPK_ACT_ELU>), dim3((unsigned)blocks), dim3(64), 0, stream, net, n, x, f);
        break;
      default:
        hipLaunchKernelGGL((eval_kernel<H, SPK_ACT_SIN>), dim3((unsigned)blocks), dim3(64), 0, stream, net, n, x, f);
        break;
    }
    return hipGetLastError();
  }
}

spk_status launch_eval(const spk_net* net, int64_t n, const float* x, float* f, hipStream_t stream, int num_cus) {
  hipError_t e;
  switch (net->dev.H) {
    case 32: e = launch_eval_h<32>(net->dev, n, x, f, stream, num_cus); break;
    case 64: e = launch_eval_h<64>(net->dev, n, x, f, stream, num_cus); break;
    case 128: e = launch_eval_h<128>(net->dev, n, x, f, stream, num_cus); break;
    case 256: e = launch_eval_h<256>(net->dev, n, x, f, stream, num_cus); break;
    default: return SPK_E_UNSUPPORTED;
  }
  return e == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
