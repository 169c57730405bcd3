// Intersection of two implicit shapes (Section 4.9) on gfx950: octree rounds
// over the cells that may hold a common point of the solids {f < 0} and
// {g < 0}.  Both networks bound every frontier cell (two bound launches);
// one kernel then combines the labels: a cell with either function POSITIVE
// is dropped, a cell with both NEGATIVE is a witness (the smallest code is
// kept by an atomic minimum), other cells emit their 8 children (or count as
// undecided at the maximum level), compacted with one atomic per wave.
#include "spk_impl.h"

namespace spk {

__global__ __launch_bounds__(256) void ix_combine_kernel(IxRound X) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < X.n; base += stride) {
    const int64_t i = base + lane;
    const bool in = i < X.n;
    const uint8_t a = in ? X.lab_f[i] : (uint8_t)SPK_POSITIVE;
    const uint8_t b = in ? X.lab_g[i] : (uint8_t)SPK_POSITIVE;
    const bool both_neg = a == SPK_NEGATIVE && b == SPK_NEGATIVE;
    const bool keep = !both_neg && a != SPK_POSITIVE && b != SPK_POSITIVE;
    const uint64_t code = in ? X.cells[i] : 0ull;
    if (both_neg) {
      atomicMin(&X.counts[2], (unsigned long long)code);
      atomicAdd(&X.counts[3], 1ull);
    }
    const unsigned long long mk = __ballot(keep);
    const int nk = __popcll(mk);
    unsigned long long off = 0ull;
    if (lane == 0 && nk) off = atomicAdd(&X.counts[X.at_max ? 1 : 0], (unsigned long long)(X.at_max ? nk : 8 * nk));
    off = __shfl(off, 0, 64);
    if (keep && !X.at_max) {
      const int64_t pre = __popcll(mk & below);
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int64_t p = (int64_t)off + 8 * pre + o;
        if (p < X.cap) X.children[p] = (code << 3) | (uint64_t)o;
      }
    }
  }
}

// counts: [0] children, [1] undecided cells at the maximum level, [2] the
// smallest witness code (all ones: none), [3] witnesses
__global__ void ix_reset_kernel(unsigned long long* counts) {
  if (threadIdx.x < 4) counts[threadIdx.x] = threadIdx.x == 2 ? ~0ull : 0ull;
}

spk_status launch_ix_round(const IxRound& X, hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(ix_reset_kernel, dim3(1), dim3(64), 0, stream, X.counts);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  if (X.n <= 0) return SPK_OK;
  int64_t blocks = (X.n + 255) / 256;
  if (blocks > (int64_t)num_cus * 8) blocks = (int64_t)num_cus * 8;
  hipLaunchKernelGGL(ix_combine_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
