// Empty spheres (Section 4.4) on gfx950: rounds over the live queries.  Each
// round bounds f over the cube [p - r, p + r]^3 of every live query (rounded
// outwards to FP32, so it contains the ball of radius r) with the box bound
// kernel; a classified cube answers the query with radius r, otherwise r is
// halved, and a query whose radius would fall below r_min ends with 0.  The
// live list is compacted with one atomic counter per round.
#include "spk_impl.h"

namespace spk {

__global__ __launch_bounds__(256) void es_init_kernel(EsRound E) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E.n) return;
  E.cur[i] = (int64_t)i;
  E.r_cur[i] = E.r0;
  E.radius[i] = 0.0f;
  E.label[i] = SPK_UNKNOWN;
}

__device__ __forceinline__ float down_f(double v) {
  const float f = (float)v;
  return ((double)f > v) ? __uint_as_float(f > 0.0f ? __float_as_uint(f) - 1u
                                                    : (f == 0.0f ? 0x80000001u : __float_as_uint(f) + 1u))
                         : f;
}
__device__ __forceinline__ float up_f(double v) { return -down_f(-v); }

__global__ __launch_bounds__(256) void es_boxes_kernel(EsRound E, int64_t m) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t i = E.cur[j];
  const double r = (double)E.r_cur[j];
  for (int d = 0; d < 3; ++d) {
    const double c = (double)E.p[3 * i + d];
    E.box_lo[3 * j + d] = down_f(c - r);
    E.box_hi[3 * j + d] = up_f(c + r);
  }
}

__global__ __launch_bounds__(256) void es_update_kernel(EsRound E, int64_t m) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t i = E.cur[j];
  const float r = E.r_cur[j];
  const uint8_t lab = E.lab_cur[j];
  if (lab != SPK_UNKNOWN) {
    E.radius[i] = r;
    E.label[i] = lab;
    return;
  }
  const float rn = 0.5f * r;
  if (!(rn >= E.r_min)) return;   // radius 0, UNKNOWN (written at init)
  const unsigned long long k = atomicAdd(E.count, 1ull);
  E.next[k] = i;
  E.r_next[k] = rn;
}

__global__ void es_zero_kernel(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

static inline unsigned grid256(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

spk_status launch_es_init(const EsRound& E, hipStream_t stream) {
  hipLaunchKernelGGL(es_init_kernel, dim3(grid256(E.n)), dim3(256), 0, stream, E);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_es_boxes(const EsRound& E, int64_t m, hipStream_t stream) {
  hipLaunchKernelGGL(es_boxes_kernel, dim3(grid256(m)), dim3(256), 0, stream, E, m);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_es_update(const EsRound& E, int64_t m, hipStream_t stream) {
  hipLaunchKernelGGL(es_zero_kernel, dim3(1), dim3(64), 0, stream, E.count);
  hipLaunchKernelGGL(es_update_kernel, dim3(grid256(m)), dim3(256), 0, stream, E, m);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
