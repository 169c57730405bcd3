// Sampling in leaf cells (surface sampling, Section 4.6; bulk properties,
// Section 4.8) on gfx950.  Sample i takes outputs 4i .. 4i+3 of the splitmix64
// generator (Steele, Lea and Flood, 2014) seeded with `seed`: the first picks
// the leaf (modulo the leaf count; all leaves of one level have the same
// size), the others give 24-bit uniform offsets in [0, 1) per axis.  The
// points are evaluated, and those with |f| < band are compacted with one
// atomic per wave; the accepted samples with f < 0 are counted.
#include "spk_impl.h"

namespace spk {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  // the k-th output (k = 0, 1, ...) of the generator seeded with `seed`
  uint64_t z = seed + (k + 1ull) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void sample_points_kernel(SampleJob J, int64_t i0, int64_t m, float* pts) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t i = (uint64_t)(i0 + t);
    const uint64_t leaf = splitmix64_at(J.seed, 4ull * i) % (uint64_t)J.n_leaves;
    float lo[3], hi[3];
    cell_box(J.leaves[leaf], J.level, J.dom_lo, J.dom_hi, lo, hi);
    for (int d = 0; d < 3; ++d) {
      const float u = (float)(splitmix64_at(J.seed, 4ull * i + 1ull + (uint64_t)d) >> 40) * 5.9604644775390625e-08f;
      pts[3 * t + d] = lo[d] + u * (hi[d] - lo[d]);
    }
  }
}

__global__ __launch_bounds__(256) void sample_accept_kernel(SampleJob J, int64_t m, const float* pts,
                                                            const float* vals) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < m; base += stride) {
    const int64_t t = base + lane;
    const float f = t < m ? vals[t] : 0.0f;
    const bool ok = t < m && fabsf(f) < J.band;
    const unsigned long long ma = __ballot(ok);
    const unsigned long long mb = __ballot(ok && f < 0.0f);
    unsigned long long off = 0ull;
    if (lane == 0) {
      if (ma) off = atomicAdd(&J.counts[0], (unsigned long long)__popcll(ma));
      if (mb) atomicAdd(&J.counts[1], (unsigned long long)__popcll(mb));
    }
    off = __shfl(off, 0, 64);
    if (ok) {
      const int64_t k = (int64_t)off + __popcll(ma & below);
      if (k < J.cap) {
        for (int d = 0; d < 3; ++d) J.points[3 * k + d] = pts[3 * t + d];
        if (J.f) J.f[k] = f;
      }
    }
  }
}

static inline unsigned grid_s(int64_t n, int num_cus) {
  int64_t b = (n + 255) / 256;
  if (b > (int64_t)num_cus * 16) b = (int64_t)num_cus * 16;
  return (unsigned)(b > 0 ? b : 1);
}

spk_status launch_sample_chunk(const spk_net* net, const SampleJob& J, int64_t i0, int64_t m, float* pts, float* vals,
                               hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(sample_points_kernel, dim3(grid_s(m, num_cus)), dim3(256), 0, stream, J, i0, m, pts);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  spk_status st = launch_eval(net, m, pts, vals, stream, num_cus);
  if (st != SPK_OK) return st;
  hipLaunchKernelGGL(sample_accept_kernel, dim3(grid_s(m, num_cus)), dim3(256), 0, stream, J, m, pts, vals);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
