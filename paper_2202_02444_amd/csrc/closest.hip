// Closest point on the level set (Section 4.10) for many query points, as
// level-synchronous rounds over (query, octree cell) pairs.
//
// The paper descends the lazily classified octree best-first per query.  On
// the GPU every query advances one level per round instead:
//   1. the bound kernel classifies every frontier cell (Procedure 1);
//   2. f is evaluated at the six face centers of every cell;
//   3. an UNKNOWN cell whose face centers show both signs spans the level set:
//      the query's distance bound drops to the farthest distance from the
//      query to the cell (atomic minimum), and a cell attaining the bound
//      becomes the candidate point (its center);
//   4. UNKNOWN cells below the maximum level emit the children that could
//      still hold a closer point (minimum distance below the current bound).
// A cell whose minimum distance is not below the bound is skipped; it could
// not lower the bound (its farthest distance is at least its minimum), so the
// final bound equals that of the best-first order, which only visits cells in
// a different order.
//
// Queries near the same stretch of surface share most of their frontier
// cells, and a cell's bound and face values do not depend on the query: on
// large rounds the distinct cells are found (radix sort of the codes, then
// unique), classified and evaluated once, and every (query, cell) item reads
// its cell's results by binary search.
#include <hipcub/hipcub.hpp>

#include "spk_impl.h"

namespace spk {

__device__ __forceinline__ void cp_cell_box(uint64_t code, int level, const CpLevel& L, float (&lo)[3],
                                            float (&hi)[3]) {
  cell_box(code, level, L.dom_lo, L.dom_hi, lo, hi);
}

__device__ __forceinline__ float min_dist(const float (&q)[3], const float (&lo)[3], const float (&hi)[3]) {
  float s = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float v = fmaxf(fmaxf(lo[d] - q[d], q[d] - hi[d]), 0.0f);
    s = fmaf(v, v, s);
  }
  return sqrtf(s);
}

__device__ __forceinline__ float max_dist(const float (&q)[3], const float (&lo)[3], const float (&hi)[3]) {
  float s = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float v = fmaxf(fabsf(q[d] - lo[d]), fabsf(q[d] - hi[d]));
    s = fmaf(v, v, s);
  }
  return sqrtf(s);
}

__device__ __forceinline__ void load_q(const CpLevel& L, uint32_t qi, float (&q)[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) q[d] = L.q[3 * (size_t)qi + d];
}

__global__ __launch_bounds__(256) void cp_init_kernel(int64_t n, uint64_t* codes, uint32_t* qidx, unsigned* best,
                                                      float* point) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    codes[i] = 0ull;
    qidx[i] = (uint32_t)i;
    best[i] = 0x7f800000u;   // +inf
#pragma unroll
    for (int d = 0; d < 3; ++d) point[3 * i + d] = __int_as_float(0x7fc00000);
  }
}

// Face centers of every frontier cell.
__global__ __launch_bounds__(256) void cp_faces_kernel(CpLevel L) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.m; i += (int64_t)gridDim.x * blockDim.x) {
    float lo[3], hi[3];
    cp_cell_box(L.codes[i], L.level, L, lo, hi);
    write_faces(lo, hi, L.fpts + 18 * i);
  }
}

// Whether frontier item i is live (not pruned), and if so whether it spans.
__device__ __forceinline__ bool cp_live(const CpLevel& L, int64_t i, float (&q)[3], float (&lo)[3], float (&hi)[3]) {
  const uint32_t qi = L.qidx[i];
  load_q(L, qi, q);
  cp_cell_box(L.codes[i], L.level, L, lo, hi);
  const float bound = __uint_as_float(L.best[qi]);
  return L.label[i] == SPK_UNKNOWN && min_dist(q, lo, hi) < bound;
}

__device__ __forceinline__ bool cp_spans(const CpLevel& L, int64_t i) { return spans6(L.fvals + 6 * i); }

__global__ __launch_bounds__(256) void cp_update_kernel(CpLevel L) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.m; i += (int64_t)gridDim.x * blockDim.x) {
    float q[3], lo[3], hi[3];
    if (!cp_live(L, i, q, lo, hi) || !cp_spans(L, i)) continue;
    // distances are >= 0, so their bit patterns order like the values
    atomicMin(&L.best[L.qidx[i]], __float_as_uint(max_dist(q, lo, hi)));
  }
}

// After cp_update: a spanning cell that attains its query's bound writes its
// center as the candidate (any one of equal cells).  Liveness is judged
// against the bound before this round's update, like in cp_update.
__global__ __launch_bounds__(256) void cp_point_kernel(CpLevel L) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.m; i += (int64_t)gridDim.x * blockDim.x) {
    if (L.label[i] != SPK_UNKNOWN || !cp_spans(L, i)) continue;
    const uint32_t qi = L.qidx[i];
    float q[3], lo[3], hi[3];
    load_q(L, qi, q);
    cp_cell_box(L.codes[i], L.level, L, lo, hi);
    if (__float_as_uint(max_dist(q, lo, hi)) != L.best[qi]) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) L.point[3 * (size_t)qi + d] = 0.5f * (lo[d] + hi[d]);
  }
}

__global__ void cp_zero_kernel(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

// Children of live UNKNOWN cells whose minimum distance is below the bound,
// compacted with one atomic per wave.
__global__ __launch_bounds__(256) void cp_expand_kernel(CpLevel L) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < L.m; base += stride) {
    const int64_t i = base + lane;
    uint32_t keep = 0u;
    uint64_t code = 0ull;
    uint32_t qi = 0u;
    if (i < L.m) {
      float q[3], lo[3], hi[3];
      if (cp_live(L, i, q, lo, hi)) {
        code = L.codes[i];
        qi = L.qidx[i];
        const float bound = __uint_as_float(L.best[qi]);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          float cl[3], chh[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const float mid = 0.5f * (lo[d] + hi[d]);
            const bool up = (o >> d) & 1;
            cl[d] = up ? mid : lo[d];
            chh[d] = up ? hi[d] : mid;
          }
          if (min_dist(q, cl, chh) < bound) keep |= 1u << o;
        }
      }
    }
    const int cnt = __popc(keep);
    // wave prefix sum of the per-lane child counts
    int incl = cnt;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
      const int v = __shfl_up(incl, s, 64);
      if (lane >= s) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    unsigned long long off = 0ull;
    if (lane == 63 && total > 0) off = atomicAdd(L.ncount, (unsigned long long)total);
    off = __shfl(off, 63, 64);
    int64_t p = (int64_t)off + incl - cnt;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      if ((keep >> o) & 1u) {
        if (p < L.cap) {
          L.ncodes[p] = (code << 3) | (uint64_t)o;
          L.nqidx[p] = qi;
        }
        ++p;
      }
    }
  }
}

__global__ __launch_bounds__(256) void cp_finish_kernel(int64_t n, const float* q, const unsigned* best,
                                                        float* point, float* dist, float* best_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float b = __uint_as_float(best[i]);
    if (best_out) best_out[i] = b;
    float s = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float v = point[3 * i + d] - q[3 * i + d];
      s = fmaf(v, v, s);
    }
    const float r = sqrtf(s);
    if (dist) dist[i] = isfinite(b) ? r : INFINITY;
  }
}

// ---------------------------------------------------------------------------
// Seeding descent.  Before the level rounds every query walks down from the
// root one cell per level: of the current cell's 8 children it enters the
// nearest (minimum distance) UNKNOWN child that spans the surface, else the
// nearest UNKNOWN child, and it lowers its bound by the farthest distance to
// the best spanning UNKNOWN child.  The walk stops when no child is UNKNOWN
// or the nearest one is not closer than the bound.
//
// Every cell that lowers the seed is a spanning UNKNOWN cell whose ancestors
// are UNKNOWN (the path), tested with the same face centers, evaluation and
// distance functions as the level rounds.  The rounds reach such a cell
// unless a bound below its farthest distance prunes an ancestor first, so
// with or without the seed they end with the same bound: the seed only prunes
// cells that could not lower it.
// ---------------------------------------------------------------------------
constexpr uint64_t kDead = ~0ull;

__global__ __launch_bounds__(256) void cp_dive_init_kernel(int64_t n, uint64_t* cur) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    cur[i] = 0ull;   // the root
}

__global__ __launch_bounds__(256) void cp_dive_children_kernel(CpDive D) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 8 * D.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t c = D.cur[i >> 3];
    // a stopped query still fills its 8 slots (with a valid cell) so that
    // every label and face value read later is written
    const uint64_t code = (c == kDead) ? 0ull : ((c << 3) | (uint64_t)(i & 7));
    D.codes[i] = code;
    float lo[3], hi[3];
    cell_box(code, D.level, D.dom_lo, D.dom_hi, lo, hi);
    write_faces(lo, hi, D.fpts + 18 * i);
  }
}

__global__ __launch_bounds__(256) void cp_dive_pick_kernel(CpDive D) {
  for (int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; qi < D.n; qi += (int64_t)gridDim.x * blockDim.x) {
    if (D.cur[qi] == kDead) continue;
    float q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) q[d] = D.q[3 * qi + d];
    int pick = -1, best_span = -1;
    bool pick_spans = false;
    float pick_min = INFINITY;
    unsigned bmax = 0xffffffffu;
    for (int o = 0; o < 8; ++o) {
      const int64_t i = 8 * qi + o;
      if (D.label[i] != SPK_UNKNOWN) continue;
      float lo[3], hi[3];
      cell_box(D.codes[i], D.level, D.dom_lo, D.dom_hi, lo, hi);
      const bool sp = spans6(D.fvals + 6 * i);
      const float md = min_dist(q, lo, hi);
      if (pick < 0 || (sp && !pick_spans) || (sp == pick_spans && md < pick_min)) {
        pick = o;
        pick_spans = sp;
        pick_min = md;
      }
      if (sp) {
        const unsigned b = __float_as_uint(max_dist(q, lo, hi));
        if (b < bmax) {
          bmax = b;
          best_span = o;
        }
      }
    }
    if (best_span >= 0 && bmax < D.best[qi]) {
      D.best[qi] = bmax;
      float lo[3], hi[3];
      cell_box(D.codes[8 * qi + best_span], D.level, D.dom_lo, D.dom_hi, lo, hi);
#pragma unroll
      for (int d = 0; d < 3; ++d) D.point[3 * qi + d] = 0.5f * (lo[d] + hi[d]);
    }
    const bool go = pick >= 0 && pick_min < __uint_as_float(D.best[qi]);
    D.cur[qi] = go ? D.codes[8 * qi + pick] : kDead;
  }
}

static inline unsigned grid_for(int64_t n, int num_cus) {
  int64_t b = (n + 255) / 256;
  if (b > (int64_t)num_cus * 8) b = (int64_t)num_cus * 8;
  if (b < 1) b = 1;
  return (unsigned)b;
}

spk_status launch_cp_init(int64_t n, uint64_t* codes, uint32_t* qidx, unsigned* best, float* point,
                          hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(cp_init_kernel, dim3(grid_for(n, num_cus)), dim3(256), 0, stream, n, codes, qidx, best, point);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

// Item i reads the label and face values of its cell from the distinct
// cells' arrays (ucodes sorted ascending, every item's code among them).
__global__ __launch_bounds__(256) void cp_gather_kernel(const uint64_t* codes, int64_t m, const uint64_t* ucodes,
                                                        int64_t nu, const uint8_t* ulabel, const float* ufvals,
                                                        uint8_t* label, float* fvals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t c = codes[i];
    int64_t lo = 0, hi = nu - 1;   // ucodes[lo] <= c <= ucodes[hi]
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ucodes[mid] < c)
        lo = mid + 1;
      else
        hi = mid;
    }
    label[i] = ulabel[lo];
#pragma unroll
    for (int f = 0; f < 6; ++f) fvals[6 * i + f] = ufvals[6 * lo + f];
  }
}

size_t cp_dedup_temp_bytes(int64_t m) {
  size_t a = 0, b = 0;
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, a, (const uint64_t*)nullptr, (uint64_t*)nullptr, (int)m);
  (void)hipcub::DeviceSelect::Unique(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr, (int64_t*)nullptr,
                                     (int)m);
  return (a > b ? a : b) + 256;
}

spk_status launch_cp_dedup(const uint64_t* codes, uint64_t* sorted, uint64_t* ucodes, int64_t* nu, int64_t m,
                           int level, void* temp, size_t temp_bytes, hipStream_t stream) {
  if (m <= 0 || m > (int64_t)0x7fffffff) return SPK_E_INVAL;
  size_t tb = temp_bytes;
  // the codes of level `level` occupy the low 3 level bits
  const int end_bit = level > 0 ? 3 * level : 1;
  if (hipcub::DeviceRadixSort::SortKeys(temp, tb, codes, sorted, (int)m, 0, end_bit, stream) != hipSuccess)
    return SPK_E_DEVICE;
  tb = temp_bytes;
  if (hipcub::DeviceSelect::Unique(temp, tb, sorted, ucodes, nu, (int)m, stream) != hipSuccess) return SPK_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_cp_shared(const spk_net* net, const CpLevel& U, const uint64_t* codes, int64_t m,
                            const uint8_t* ulabel, float* ufvals, uint8_t* label, float* fvals, hipStream_t stream,
                            int num_cus) {
  hipLaunchKernelGGL(cp_faces_kernel, dim3(grid_for(U.m, num_cus)), dim3(256), 0, stream, U);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  spk_status st = launch_eval(net, 6 * U.m, U.fpts, ufvals, stream, num_cus);
  if (st != SPK_OK) return st;
  hipLaunchKernelGGL(cp_gather_kernel, dim3(grid_for(m, num_cus)), dim3(256), 0, stream, codes, m, U.codes, U.m,
                     ulabel, ufvals, label, fvals);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_cp_round(const spk_net* net, const CpLevel& L, hipStream_t stream, int num_cus) {
  const unsigned g = grid_for(L.m, num_cus);
  if (!L.shared) {
    hipLaunchKernelGGL(cp_faces_kernel, dim3(g), dim3(256), 0, stream, L);
    if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
    spk_status st = launch_eval(net, 6 * L.m, L.fpts, L.fvals, stream, num_cus);
    if (st != SPK_OK) return st;
  }
  hipLaunchKernelGGL(cp_update_kernel, dim3(g), dim3(256), 0, stream, L);
  hipLaunchKernelGGL(cp_point_kernel, dim3(g), dim3(256), 0, stream, L);
  if (!L.at_max) {
    hipLaunchKernelGGL(cp_zero_kernel, dim3(1), dim3(64), 0, stream, L.ncount);
    hipLaunchKernelGGL(cp_expand_kernel, dim3(g), dim3(256), 0, stream, L);
  }
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_cp_dive_init(int64_t n, uint64_t* cur, hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(cp_dive_init_kernel, dim3(grid_for(n, num_cus)), dim3(256), 0, stream, n, cur);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_cp_dive_children(const CpDive& D, hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(cp_dive_children_kernel, dim3(grid_for(8 * D.n, num_cus)), dim3(256), 0, stream, D);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_cp_dive_pick(const CpDive& D, hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(cp_dive_pick_kernel, dim3(grid_for(D.n, num_cus)), dim3(256), 0, stream, D);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_cp_finish(int64_t n, const float* q, const unsigned* best, float* point, float* dist,
                            float* best_out, hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(cp_finish_kernel, dim3(grid_for(n, num_cus)), dim3(256), 0, stream, n, q, best, point, dist,
                     best_out);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
