// Frontier compaction of one BuildSpatialTree round (Procedure 3 run in
// parallel rounds, Section 4.5): UNKNOWN cells below the maximum level emit
// their 8 children, UNKNOWN cells at the maximum level go to the leaf list,
// POSITIVE/NEGATIVE cells are counted.  Wave-level ballot + prefix count, one
// atomic per wave and output list.
#include "spk_impl.h"

namespace spk {

__global__ void zero_counts_kernel(unsigned long long* counts) {
  if (threadIdx.x < 4) counts[threadIdx.x] = 0ull;
}

// One wave's chunk of 64 consecutive cells [base, base + 64) of a round.
__device__ __forceinline__ void compact_chunk(const uint8_t* __restrict__ labels, const uint64_t* __restrict__ cells,
                                              int64_t n, int at_max, uint64_t* __restrict__ children,
                                              int64_t cap_children, uint64_t* __restrict__ leaves, int64_t cap_leaves,
                                              unsigned long long* counts, int64_t base, int lane) {
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t i = base + lane;
  const bool in = i < n;
  const uint8_t lab = in ? labels[i] : (uint8_t)255;
  const bool unk = lab == SPK_UNKNOWN;
  // converged cells (the delta test) and UNKNOWN cells at the maximum level
  // are leaves; other UNKNOWN cells split
  const bool to_leaf = lab == kConverged || (at_max && unk);
  const bool to_kids = !at_max && unk;
  const unsigned long long mk = __ballot(to_kids);
  const unsigned long long ml = __ballot(to_leaf);
  const unsigned long long mp = __ballot(lab == SPK_POSITIVE);
  const unsigned long long mn = __ballot(lab == SPK_NEGATIVE);
  unsigned long long offk = 0ull, offl = 0ull;
  if (lane == 0) {
    if (mk) offk = atomicAdd(&counts[0], 8ull * (unsigned long long)__popcll(mk));
    if (ml) offl = atomicAdd(&counts[1], (unsigned long long)__popcll(ml));
    if (mp) atomicAdd(&counts[2], (unsigned long long)__popcll(mp));
    if (mn) atomicAdd(&counts[3], (unsigned long long)__popcll(mn));
  }
  offk = __shfl(offk, 0, 64);
  offl = __shfl(offl, 0, 64);
  if (to_leaf) {
    const int64_t p = (int64_t)offl + __popcll(ml & below);
    if (p < cap_leaves) leaves[p] = cells[i];
  } else if (to_kids) {
    const int64_t pre = __popcll(mk & below);
    const uint64_t code = cells[i];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int64_t p = (int64_t)offk + 8 * pre + o;
      if (p < cap_children) children[p] = (code << 3) | (uint64_t)o;
    }
  }
}

// The convergence test (Procedure 3, small cells): face centers of every
// cell, then UNKNOWN cells whose face values show both signs become
// kConverged.
__global__ __launch_bounds__(256) void converge_faces_kernel(const uint64_t* cells, int64_t n, int level, CellDom dom,
                                                             float* fpts) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float lo[3], hi[3];
    cell_box(cells[i], level, dom.lo, dom.hi, lo, hi);
    write_faces(lo, hi, fpts + 18 * i);
  }
}

__global__ __launch_bounds__(256) void converge_mark_kernel(uint8_t* labels, int64_t n, const float* fvals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (labels[i] == SPK_UNKNOWN && spans6(fvals + 6 * i)) labels[i] = kConverged;
}

spk_status launch_converge(const spk_net* net, uint8_t* labels, const uint64_t* cells, int64_t n, int level,
                           const float (&dom_lo)[3], const float (&dom_hi)[3], float* fpts, float* fvals,
                           hipStream_t stream, int num_cus) {
  if (n <= 0) return SPK_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)num_cus * 8) blocks = (int64_t)num_cus * 8;
  CellDom dom;
  for (int d = 0; d < 3; ++d) {
    dom.lo[d] = dom_lo[d];
    dom.hi[d] = dom_hi[d];
  }
  hipLaunchKernelGGL(converge_faces_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, cells, n, level, dom, fpts);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  spk_status st = launch_eval(net, 6 * n, fpts, fvals, stream, num_cus);
  if (st != SPK_OK) return st;
  hipLaunchKernelGGL(converge_mark_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, labels, n, fvals);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

__global__ __launch_bounds__(256) void compact_kernel(const uint8_t* __restrict__ labels,
                                                      const uint64_t* __restrict__ cells, int64_t n, int at_max,
                                                      uint64_t* __restrict__ children, int64_t cap_children,
                                                      uint64_t* __restrict__ leaves, int64_t cap_leaves,
                                                      unsigned long long* counts) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride)
    compact_chunk(labels, cells, n, at_max, children, cap_children, leaves, cap_leaves, counts, base, lane);
}

// The rounds of many networks at once (the batched graph): wave chunks are
// numbered across the items by the prefix sums of their chunk counts.
__global__ __launch_bounds__(256) void batch_compact_kernel(const CompactItem* items, const int64_t* prefix,
                                                            int n_items) {
  const int lane = threadIdx.x & 63;
  const int64_t total = prefix[n_items];
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t cid = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); cid < total; cid += waves) {
    int lo = 0, hi = n_items;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (prefix[mid] <= cid) lo = mid;
      else hi = mid;
    }
    const CompactItem it = items[lo];
    compact_chunk(it.labels, it.cells, it.n, it.at_max, it.children, it.cap_children, it.leaves, it.cap_leaves,
                  it.counts, 64 * (cid - prefix[lo]), lane);
  }
}

__global__ void batch_counts_zero_kernel(const CompactItem* items, int n_items) {
  for (int i = threadIdx.x; i < n_items; i += blockDim.x)
    if (items[i].counts != nullptr)
      for (int c = 0; c < 4; ++c) items[i].counts[c] = 0ull;
}

// Device status of a round (spk_device_status layout: nospc at byte 8, the
// required capacities at bytes 16 and 24): one thread compares the round's
// counts with its capacities after the compaction.
__global__ void round_status_kernel(const unsigned long long* counts, int64_t cap_children, int64_t cap_leaves,
                                    unsigned char* status) {
  if (threadIdx.x != 0) return;
  const unsigned long long nc = counts[0], nl = counts[1];
  if (nc > (unsigned long long)cap_children || nl > (unsigned long long)cap_leaves) {
    *(int*)(status + 8) = 1;
    atomicMax((unsigned long long*)(status + 16), nc);
    atomicMax((unsigned long long*)(status + 24), nl);
  }
}

hipError_t launch_batch_compact(const CompactItem* items, const int64_t* prefix, int n_items, int blocks,
                                hipStream_t stream) {
  hipLaunchKernelGGL(batch_counts_zero_kernel, dim3(1), dim3(256), 0, stream, items, n_items);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_compact_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, items, prefix, n_items);
  return hipGetLastError();
}

spk_status launch_compact(const uint8_t* labels, const uint64_t* cells, int64_t n, bool at_max, uint64_t* children,
                          int64_t cap_children, uint64_t* leaves, int64_t cap_leaves, int64_t* counts, void* status,
                          hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, stream, (unsigned long long*)counts);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  if (n <= 0) return SPK_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)num_cus * 8) blocks = (int64_t)num_cus * 8;
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, labels, cells, n, at_max ? 1 : 0,
                     children, cap_children, leaves, cap_leaves, (unsigned long long*)counts);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  if (status != nullptr) {
    hipLaunchKernelGGL(round_status_kernel, dim3(1), dim3(64), 0, stream, (const unsigned long long*)counts,
                       cap_children, cap_leaves, (unsigned char*)status);
    if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  }
  return SPK_OK;
}

}  // namespace spk
