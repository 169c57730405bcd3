// Frustum ray casting (Section 4.3; Appendix B) on gfx950: device side.
//
// The image is covered by a grid of coarse frusta (rectangles of pixels that
// share the eye).  Every round bounds f over one oriented box per live
// frustum (its part between distances t and t + sigma along the rays) with
// the general-box bound kernel, then advances, shrinks or splits the frusta:
//   * the box misses the domain [-1,1]^3 or f is bounded away from zero on
//     it: t += safety sigma, sigma grows (a frustum past the domain's far
//     side is finished: all its rays miss);
//   * otherwise sigma shrinks, and a frustum wider than 2 sigma at distance
//     t + sigma along an image direction (or with sigma below delta) splits
//     in half along the wider direction; a single pixel is handed off to
//     Procedure 2 from its current t.
// The frusta of a round are disjoint pixel sets, so a list of width x height
// entries always holds the next round; the lists are compacted with one
// atomic counter.
#include "spk_impl.h"

namespace spk {

namespace {

__device__ __forceinline__ double tan_x_of(const FrCam& c, double px) {
  return (2.0 * (px + 0.5) / (double)c.width - 1.0) * c.tan_x;
}
__device__ __forceinline__ double tan_y_of(const FrCam& c, double py) {
  return (1.0 - 2.0 * (py + 0.5) / (double)c.height) * c.tan_y;
}

__device__ __forceinline__ double near0(double lo, double hi) {
  return (lo <= 0.0 && hi >= 0.0) ? 0.0 : fmin(fabs(lo), fabs(hi));
}

// Extremes of s g over s in [t, s1] and the rectangle, for one lateral
// coordinate g = a / sqrt(1 + a^2 + b^2) (a the coordinate's own tangent, b
// the other's): monotone in a; for fixed a its magnitude falls with b^2.
__device__ __forceinline__ void lateral(double alo, double ahi, double bmin2, double bmax2, double t, double s1,
                                        double& cmin, double& cmax) {
  const double gmax = ahi / sqrt(1.0 + ahi * ahi + (ahi >= 0.0 ? bmin2 : bmax2));
  const double gmin = alo / sqrt(1.0 + alo * alo + (alo <= 0.0 ? bmin2 : bmax2));
  cmax = gmax >= 0.0 ? s1 * gmax : t * gmax;
  cmin = gmin <= 0.0 ? s1 * gmin : t * gmin;
}

}  // namespace

__global__ __launch_bounds__(256) void fr_init_kernel(FrRound R, int tiles_x, int tiles_y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tiles_x * tiles_y) return;
  const int tx = i % tiles_x, ty = i / tiles_x;
  Frustum f;
  f.x0 = (int)(((int64_t)tx * R.cam.width + tiles_x / 2) / tiles_x);
  f.x1 = (int)(((int64_t)(tx + 1) * R.cam.width + tiles_x / 2) / tiles_x);
  f.y0 = (int)(((int64_t)ty * R.cam.height + tiles_y / 2) / tiles_y);
  f.y1 = (int)(((int64_t)(ty + 1) * R.cam.height + tiles_y / 2) / tiles_y);
  f.t = R.t0;
  f.sigma = R.sigma0;
  f.steps = 0;
  f.pad = 0;
  R.cur[i] = f;
}

// The oriented box of each live frustum in the camera frame, rounded to FP32
// and widened by `margin` (the FP32 rounding of the box, camera vectors that
// are orthonormal only to 1e-6, and the FP32 rays of the handed-off pixels),
// plus whether it misses the domain.
__global__ __launch_bounds__(256) void fr_box_kernel(FrRound R, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const Frustum f = R.cur[i];
  const FrCam& c = R.cam;
  const double t = (double)f.t, s1 = (double)f.t + (double)f.sigma;
  const double xa = tan_x_of(c, f.x0), xb = tan_x_of(c, f.x1 - 1);
  const double ya = tan_y_of(c, f.y1 - 1), yb = tan_y_of(c, f.y0);
  const double xlo = fmin(xa, xb), xhi = fmax(xa, xb), ylo = fmin(ya, yb), yhi = fmax(ya, yb);
  const double mx = near0(xlo, xhi), my = near0(ylo, yhi);
  const double mx2 = mx * mx, my2 = my * my;
  const double Mx2 = fmax(xlo * xlo, xhi * xhi), My2 = fmax(ylo * ylo, yhi * yhi);
  double lo[3], hi[3];
  lo[0] = t / sqrt(1.0 + Mx2 + My2);
  hi[0] = s1 / sqrt(1.0 + mx2 + my2);   // the spherical front: nearest the axis
  lateral(xlo, xhi, my2, My2, t, s1, lo[1], hi[1]);
  lateral(ylo, yhi, mx2, Mx2, t, s1, lo[2], hi[2]);
  const double* A[3] = {c.F, c.Rt, c.U};
  double cen[3], half[3];
  for (int d = 0; d < 3; ++d) cen[d] = c.eye[d];
  for (int a = 0; a < 3; ++a) {
    const double mid = 0.5 * (lo[a] + hi[a]);
    half[a] = 0.5 * (hi[a] - lo[a]);
    for (int d = 0; d < 3; ++d) cen[d] += mid * A[a][d];
  }
  float c32[3];
  double dc = 0.0;
  for (int d = 0; d < 3; ++d) {
    c32[d] = (float)cen[d];
    dc += fabs(cen[d] - (double)c32[d]);
  }
  const double margin = dc + 1.0e-5 * (s1 + 1.0) + 1e-30;
  double ext[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < 3; ++a) {
    const double h = (half[a] + margin) * (1.0 + 1.0e-6);
    for (int d = 0; d < 3; ++d) {
      const float v = (float)(h * A[a][d]);
      R.axes[(9 * i + 3 * a) + d] = v;
      ext[d] += fabs((double)v);
    }
  }
  bool miss = false;
  for (int d = 0; d < 3; ++d) {
    R.center[3 * i + d] = c32[d];
    miss = miss || ((double)c32[d] - ext[d] > 1.0) || ((double)c32[d] + ext[d] < -1.0);
  }
  R.miss[i] = miss ? 1 : 0;
}

__device__ __forceinline__ void fr_emit(const FrRound& R, const Frustum& f) {
  const unsigned long long k = atomicAdd(&R.counts[0], 1ull);
  if ((int64_t)k < R.cap) R.next[k] = f;
}

// Advance, shrink, split, finish or hand off every live frustum.
__global__ __launch_bounds__(256) void fr_update_kernel(FrRound R, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  Frustum f = R.cur[i];
  f.steps += 1;
  const bool safe = R.miss[i] != 0 || R.lo[i] > 0.0f || R.hi[i] < 0.0f;
  if (safe) {
    f.t += R.p.safety * f.sigma;
    f.sigma *= R.p.eta_plus;
    if ((double)f.t < R.t_far) {
      fr_emit(R, f);
    } else {
      for (int py = f.y0; py < f.y1; ++py)
        for (int px = f.x0; px < f.x1; ++px) {
          const int64_t pix = (int64_t)py * R.cam.width + px;
          R.t_hit[pix] = INFINITY;
          if (R.iters) R.iters[pix] = f.steps;
        }
    }
    return;
  }
  f.sigma *= R.p.eta_minus;
  const int nx = f.x1 - f.x0, ny = f.y1 - f.y0;
  if (nx == 1 && ny == 1) {
    const unsigned long long k = atomicAdd(&R.counts[1], 1ull);
    if ((int64_t)k < R.cap) {
      R.hand_pix[k] = (int64_t)f.y0 * R.cam.width + f.x0;
      R.hand_t[k] = f.t;
      R.hand_steps[k] = f.steps;
    }
    return;
  }
  const FrCam& c = R.cam;
  const double s1 = (double)f.t + (double)f.sigma;
  const double wx = s1 * fabs(tan_x_of(c, f.x1 - 1) - tan_x_of(c, f.x0));
  const double wy = s1 * fabs(tan_y_of(c, f.y0) - tan_y_of(c, f.y1 - 1));
  if (fmax(wx, wy) > 2.0 * (double)f.sigma || f.sigma < R.p.delta) {
    Frustum a = f, b = f;
    if (ny == 1 || (nx > 1 && wx >= wy)) {
      const int mid = (f.x0 + f.x1) / 2;
      a.x1 = mid;
      b.x0 = mid;
    } else {
      const int mid = (f.y0 + f.y1) / 2;
      a.y1 = mid;
      b.y0 = mid;
    }
    fr_emit(R, a);
    fr_emit(R, b);
  } else {
    fr_emit(R, f);
  }
}

// Rays of the handed-off pixels from their frustum's distance t: origin
// eye + t d, direction d (FP64, rounded to FP32).
__global__ __launch_bounds__(256) void fr_rays_kernel(FrRound R, int64_t n, float* origin, float* dir) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const FrCam& c = R.cam;
  const int64_t pix = R.hand_pix[j];
  const double x = tan_x_of(c, (double)(pix % c.width)), y = tan_y_of(c, (double)(pix / c.width));
  double d[3], nn = 0.0;
  for (int k = 0; k < 3; ++k) {
    d[k] = c.F[k] + x * c.Rt[k] + y * c.U[k];
    nn += d[k] * d[k];
  }
  nn = 1.0 / sqrt(nn);
  const double t = (double)R.hand_t[j];
  for (int k = 0; k < 3; ++k) {
    d[k] *= nn;
    dir[3 * j + k] = (float)d[k];
    origin[3 * j + k] = (float)(c.eye[k] + t * d[k]);
  }
}

__global__ __launch_bounds__(256) void fr_scatter_kernel(FrRound R, int64_t n, const float* trel, const int32_t* itr) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t pix = R.hand_pix[j];
  const float tr = trel[j];
  R.t_hit[pix] = isinf(tr) ? INFINITY : R.hand_t[j] + tr;
  if (R.iters) R.iters[pix] = R.hand_steps[j] + itr[j];
  atomicAdd(&R.counts[2], (unsigned long long)itr[j]);
}

__global__ void fr_zero_kernel(unsigned long long* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

static inline unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

spk_status launch_fr_init(const FrRound& R, int tiles_x, int tiles_y, hipStream_t stream) {
  hipLaunchKernelGGL(fr_init_kernel, dim3(grid1((int64_t)tiles_x * tiles_y)), dim3(256), 0, stream, R, tiles_x,
                     tiles_y);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_fr_box(const FrRound& R, int64_t m, hipStream_t stream) {
  hipLaunchKernelGGL(fr_box_kernel, dim3(grid1(m)), dim3(256), 0, stream, R, m);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_fr_update(const FrRound& R, int64_t m, hipStream_t stream) {
  hipLaunchKernelGGL(fr_zero_kernel, dim3(1), dim3(64), 0, stream, R.counts, 1);
  hipLaunchKernelGGL(fr_update_kernel, dim3(grid1(m)), dim3(256), 0, stream, R, m);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_fr_zero(unsigned long long* counts, int n, hipStream_t stream) {
  hipLaunchKernelGGL(fr_zero_kernel, dim3(1), dim3(64), 0, stream, counts, n);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_fr_rays(const FrRound& R, int64_t n, float* origin, float* dir, hipStream_t stream) {
  hipLaunchKernelGGL(fr_rays_kernel, dim3(grid1(n)), dim3(256), 0, stream, R, n, origin, dir);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

spk_status launch_fr_scatter(const FrRound& R, int64_t n, const float* trel, const int32_t* itr, hipStream_t stream) {
  hipLaunchKernelGGL(fr_scatter_kernel, dim3(grid1(n)), dim3(256), 0, stream, R, n, trel, itr);
  return hipGetLastError() == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
