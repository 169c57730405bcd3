// Mesh extraction in the leaf cells of a frontier (Section 4.7; the dense
// evaluation of the lowest levels of Appendix B) on gfx950.  For a chunk of
// leaves: one kernel writes the grid points of every leaf (dense_levels
// further subdivisions, points dom_lo + g h with g the index on the finest
// grid, so neighbouring leaves share their face samples bit for bit), the
// evaluation kernel computes f at all of them, and one thread per grid cube
// runs marching cubes without a case table: each face joins its crossing
// edges (two crossings: one segment; four: the corners whose sign differs
// from the face's mean value are cut off), the segments close into loops,
// and each loop, walked from its lowest edge toward that edge's lower
// neighbour, is triangulated as a fan.  Triangles are appended with one
// atomic per cube.
#include "spk_impl.h"

namespace spk {

namespace {

// the 12 cube edges as corner pairs (corner c = (c & 1, c >> 1 & 1, c >> 2 & 1))
__constant__ int8_t kEdgeA[12] = {0, 2, 4, 6, 0, 1, 4, 5, 0, 1, 2, 3};
__constant__ int8_t kEdgeB[12] = {1, 3, 5, 7, 2, 3, 6, 7, 4, 5, 6, 7};
// the 6 faces: cyclic corners and the edge between corner i and corner i + 1
__constant__ int8_t kFaceC[6][4] = {{0, 2, 6, 4}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 3, 7, 6}, {0, 1, 3, 2}, {4, 5, 7, 6}};
__constant__ int8_t kFaceE[6][4] = {{4, 10, 6, 8}, {5, 11, 7, 9}, {0, 9, 2, 8}, {1, 11, 3, 10}, {0, 5, 1, 4}, {2, 7, 3, 6}};

__device__ __forceinline__ float grid_coord(const MeshJob& M, int d, int64_t g) {
  return M.dom_lo[d] + (float)g * M.h[d];
}

}  // namespace

__global__ __launch_bounds__(256) void mesh_points_kernel(MeshJob M, int64_t l0, int64_t nl, float* pts) {
  const int R = 1 << M.dense, N1 = R + 1, NV = N1 * N1 * N1;
  const int64_t total = nl * NV;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / NV;
    const int v = (int)(t - j * NV);
    const int a = v / (N1 * N1), b = (v / N1) % N1, c = v % N1;
    uint32_t idx[3] = {0u, 0u, 0u};
    const uint64_t code = M.leaves[l0 + j];
    for (int bb = 0; bb < M.level; ++bb)
      for (int d = 0; d < 3; ++d) idx[d] |= (uint32_t)((code >> (3 * bb + d)) & 1ull) << bb;
    pts[3 * t + 0] = grid_coord(M, 0, (int64_t)idx[0] * R + a);
    pts[3 * t + 1] = grid_coord(M, 1, (int64_t)idx[1] * R + b);
    pts[3 * t + 2] = grid_coord(M, 2, (int64_t)idx[2] * R + c);
  }
}

__global__ __launch_bounds__(256) void mesh_cubes_kernel(MeshJob M, int64_t l0, int64_t nl, const float* pts,
                                                         const float* vals) {
  const int R = 1 << M.dense, N1 = R + 1, NV = N1 * N1 * N1, NC = R * R * R;
  const int64_t total = nl * NC;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / NC;
    const int cube = (int)(t - j * NC);
    const int kx = cube % R, ky = (cube / R) % R, kz = cube / (R * R);
    float v[8];
    int vid[8];
    bool s[8];
    for (int c = 0; c < 8; ++c) {
      const int a = kx + (c & 1), b = ky + ((c >> 1) & 1), cc = kz + ((c >> 2) & 1);
      vid[c] = (a * N1 + b) * N1 + cc;
      v[c] = vals[j * NV + vid[c]];
      s[c] = v[c] > 0.0f;
    }
    uint32_t cross = 0u;
    for (int e = 0; e < 12; ++e)
      if (s[kEdgeA[e]] != s[kEdgeB[e]]) cross |= 1u << e;
    if (cross == 0u) continue;
    // edge points
    float pt[12][3];
    for (int e = 0; e < 12; ++e) {
      if (!((cross >> e) & 1u)) continue;
      const int a = kEdgeA[e], b = kEdgeB[e];
      const float tt = v[a] / (v[a] - v[b]);
      for (int d = 0; d < 3; ++d) {
        const float pa = pts[3 * (j * NV + vid[a]) + d], pb = pts[3 * (j * NV + vid[b]) + d];
        pt[e][d] = pa + tt * (pb - pa);
      }
    }
    // face segments: each crossing edge gets its two neighbours
    int nb[12][2], nn[12];
    for (int e = 0; e < 12; ++e) nn[e] = 0;
    for (int f = 0; f < 6; ++f) {
      int ce[4], m = 0;
      for (int i = 0; i < 4; ++i)
        if ((cross >> kFaceE[f][i]) & 1u) ce[m++] = kFaceE[f][i];
      if (m == 2) {
        nb[ce[0]][nn[ce[0]]++] = ce[1];
        nb[ce[1]][nn[ce[1]]++] = ce[0];
      } else if (m == 4) {
        const bool center = (v[kFaceC[f][0]] + v[kFaceC[f][1]] + v[kFaceC[f][2]] + v[kFaceC[f][3]]) * 0.25f > 0.0f;
        for (int i = 0; i < 4; ++i) {
          if (s[kFaceC[f][i]] == center) continue;
          const int a = kFaceE[f][(i + 3) & 3], b = kFaceE[f][i];
          nb[a][nn[a]++] = b;
          nb[b][nn[b]++] = a;
        }
      }
    }
    // loops over the crossing edges, then fans
    int order[12], starts[6], lens[6], nloops = 0, npts = 0;
    uint32_t used = 0u;
    for (int e0 = 0; e0 < 12; ++e0) {
      if (!((cross >> e0) & 1u) || ((used >> e0) & 1u)) continue;
      starts[nloops] = npts;
      int prev = e0, cur = min(nb[e0][0], nb[e0][1]);
      order[npts++] = e0;
      used |= 1u << e0;
      for (int guard = 0; cur != e0 && guard < 12 && npts < 12; ++guard) {
        order[npts++] = cur;
        used |= 1u << cur;
        const int nx = (nb[cur][0] == prev) ? nb[cur][1] : nb[cur][0];
        prev = cur;
        cur = nx;
      }
      lens[nloops] = npts - starts[nloops];
      ++nloops;
    }
    const int ntri = npts - 2 * nloops;
    const unsigned long long base = atomicAdd(M.count, (unsigned long long)ntri);
    int w = 0;
    for (int L = 0; L < nloops; ++L) {
      const int* o = order + starts[L];
      for (int i = 1; i + 1 < lens[L]; ++i, ++w) {
        const int64_t k = (int64_t)base + w;
        if (k >= M.cap) continue;
        const int tri[3] = {o[0], o[i], o[i + 1]};
        for (int q = 0; q < 3; ++q)
          for (int d = 0; d < 3; ++d) M.tris[9 * k + 3 * q + d] = pt[tri[q]][d];
        if (M.src) {
          M.src[2 * k] = (int32_t)(l0 + j);
          M.src[2 * k + 1] = cube;
        }
      }
    }
  }
}

static inline unsigned grid_of(int64_t n, int num_cus) {
  int64_t b = (n + 255) / 256;
  if (b > (int64_t)num_cus * 16) b = (int64_t)num_cus * 16;
  return (unsigned)(b > 0 ? b : 1);
}

spk_status launch_mesh_chunk(const spk_net* net, const MeshJob& M, int64_t l0, int64_t nl, float* pts, float* vals,
                             hipStream_t stream, int num_cus) {
  const int R = 1 << M.dense, N1 = R + 1;
  const int64_t npts = nl * (int64_t)(N1 * N1 * N1);
  hipLaunchKernelGGL(mesh_points_kernel, dim3(grid_of(npts, num_cus)), dim3(256), 0, stream, M, l0, nl, pts);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  spk_status st = launch_eval(net, npts, pts, vals, stream, num_cus);
  if (st != SPK_OK) return st;
  const int64_t ncubes = nl * (int64_t)(R * R * R);
  hipLaunchKernelGGL(mesh_cubes_kernel, dim3(grid_of(ncubes, num_cus)), dim3(256), 0, stream, M, l0, nl, pts, vals);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
