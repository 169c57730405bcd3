// Ray casting (Procedure 2) as a persistent work-queue kernel on gfx950.
//
// A wavefront marches BPW rays at once, one per box slot.  Each iteration is
// one affine-fixed pass of the network (the paper's ray-casting choice,
// Section 3.4) over the 1-d segment [t, t + sigma] (center p + (t + sigma/2)
// r, axis (sigma/2) r), with two passenger columns evaluating f at the
// convergence point p + (t + delta) r and at the start point.  Then, per ray:
// a sign change of f against the start returns t; otherwise the step is
// accepted (sigma* = safety sigma, sigma grows by eta_plus) when the segment
// is classified, or rejected (sigma* = 0, sigma shrinks by eta_minus), and t
// advances by max(sigma*, delta).  A finished slot takes the next ray from a
// global atomic counter; a wavefront exits when the counter is exhausted and
// all its slots are empty, so every wave terminates (at most max_iters
// iterations per ray).
#include "affine_stack.h"

namespace spk {

struct RayJob {
  int64_t n;
  const float* origin;
  const float* dir;
  float* t_hit;
  int32_t* iters;
  unsigned long long* counter;
  spk_ray_params p;
};

__global__ void zero_counter_kernel(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

// Entry/exit of o + t d in [-1,1]^3 (slab test); false if the ray misses.
__device__ __forceinline__ bool clip_cube(const float (&o)[3], const float (&d)[3], float& t_in, float& t_out) {
  float lo = 0.0f, hi = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0f) {
      if (o[a] < -1.0f || o[a] > 1.0f) return false;
    } else {
      const float inv = 1.0f / d[a];
      const float t1 = (-1.0f - o[a]) * inv, t2 = (1.0f - o[a]) * inv;
      lo = fmaxf(lo, fminf(t1, t2));
      hi = fminf(hi, fmaxf(t1, t2));
    }
  }
  t_in = lo;
  t_out = hi;
  return hi > lo;
}

template <class S, int ACT>
__global__ __launch_bounds__(64, 1) void ray_kernel(NetDev net, RayJob job) {
  __shared__ __attribute__((aligned(16))) LdsState<S> sm;
  constexpr int NS = S::NS, SEG = S::SEG, NPASS = 2;
  const int lane = threadIdx.x;
  const int bo = lane / SEG;
  const int ch = lane % SEG;
  const int segbase = bo * SEG;
  const int L = net.L;
  const spk_ray_params P = job.p;

  long long rid = -1;   // >= 0 ray index, -1 empty, -2 no rays left
  float t = 0.0f, sigma = 0.0f, f0 = 0.0f, tmax = 0.0f, base = 0.0f;
  int it = 0;
  bool first = false;
  float sp[3] = {0.0f, 0.0f, 0.0f}, dv[3] = {0.0f, 0.0f, 0.0f};

  for (;;) {
    // ---- refill: the segment's first lane takes rays until one enters the domain
    long long nr = rid;
    float np[3] = {0.0f, 0.0f, 0.0f}, nd[3] = {0.0f, 0.0f, 0.0f}, ntmax = 0.0f, nbase = 0.0f;
    if (ch == 0 && rid == -1) {
      for (;;) {
        const unsigned long long idx = atomicAdd(job.counter, 1ull);
        if (idx >= (unsigned long long)job.n) {
          nr = -2;
          break;
        }
        float o[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          o[a] = job.origin[3 * idx + a];
          d[a] = job.dir[3 * idx + a];
        }
        float t_in = 0.0f, t_out = P.t_max;
        bool inside = true;
        if (P.clip_to_domain) inside = clip_cube(o, d, t_in, t_out);
        const bool finite = isfinite(o[0]) && isfinite(o[1]) && isfinite(o[2]) && isfinite(d[0]) &&
                            isfinite(d[1]) && isfinite(d[2]);
        if (!inside || !finite || !(t_out > t_in)) {
          job.t_hit[idx] = INFINITY;
          if (job.iters) job.iters[idx] = 0;
          continue;
        }
        nr = (long long)idx;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          np[a] = o[a] + t_in * d[a];
          nd[a] = d[a];
        }
        ntmax = t_out - t_in;
        nbase = t_in;
        break;
      }
    }
    nr = __shfl(nr, segbase, 64);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      np[a] = __shfl(np[a], segbase, 64);
      nd[a] = __shfl(nd[a], segbase, 64);
    }
    ntmax = __shfl(ntmax, segbase, 64);
    nbase = __shfl(nbase, segbase, 64);
    if (rid == -1) {
      if (nr >= 0) {
        rid = nr;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          sp[a] = np[a];
          dv[a] = nd[a];
        }
        tmax = ntmax;
        base = nbase;
        t = 0.0f;
        sigma = P.sigma0;
        it = 0;
        first = true;
      } else {
        rid = -2;
      }
    }
    const bool active = rid >= 0;
    if (__ballot(active) == 0ull) break;   // every slot drained, no rays left

    // ---- one fused pass: segment bound + two point evaluations
    double cc[3];
    float ax[3][3], ein[3], pts[NPASS][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cc[a] = (double)sp[a] + ((double)t + 0.5 * (double)sigma) * (double)dv[a];
      const double v = 0.5 * (double)sigma * (double)dv[a];
      ax[0][a] = (float)v;
      ax[1][a] = 0.0f;
      ax[2][a] = 0.0f;
      ein[a] = 2.0f * kU * fabsf((float)v) + (float)(4.0 * kU64) * (float)fabs(cc[a]) + kEta;
      pts[0][a] = sp[a] + (t + P.delta) * dv[a];
      pts[1][a] = sp[a];
    }
    double xc[4];
    f4 y[NS];
    float yinf[4], e[4], u[4];
    layer0_affine<S, NPASS>(net, ch, cc, ax, ein, pts, xc, y, yinf, e);
    for (int a = 0; a < L - 1; ++a) {
      activate<S, ACT, SPK_AFFINE_FIXED, NPASS>(xc, y, yinf, e, u, 1, 0, net.cK, net.cD, net.omega0, lane,
                                                  nullptr);
      if (a == L - 2) break;
      hidden_layer<S, NPASS>(net, sm, a, xc, y, yinf, e, u, lane, false);
    }
    float pass[NPASS];
    const OutVals o = output_layer<S, NPASS>(net, xc, y, yinf, u, lane, pass);

    // ---- Procedure 2 update, identical on every lane of the segment
    if (active) {
      if (first) {
        f0 = pass[1];
        first = false;
      }
      ++it;
      const float fc = pass[0];
      if ((f0 > 0.0f) != (fc > 0.0f)) {
        if (ch == 0) {
          job.t_hit[rid] = base + t;
          if (job.iters) job.iters[rid] = it;
        }
        rid = -1;
      } else {
        float lo, hi;
        enclose(o, false, lo, hi);
        const bool safe = lo > 0.0f || hi < 0.0f;
        const float step = safe ? P.safety * sigma : 0.0f;
        sigma = safe ? sigma * P.eta_plus : sigma * P.eta_minus;
        t += fmaxf(step, P.delta);
        if (!(t < tmax) || it >= P.max_iters) {
          if (ch == 0) {
            job.t_hit[rid] = INFINITY;
            if (job.iters) job.iters[rid] = it;
          }
          rid = -1;
        }
      }
    }
  }
}

template <int H>
static hipError_t launch_rays_h(const NetDev& net, const RayJob& job, hipStream_t stream, int num_cus) {
  using S = Shape<H, 1>;
  const int64_t ngroups = (job.n + S::BPW - 1) / S::BPW;
  int64_t blocks = (int64_t)num_cus * 4;
  if (blocks > ngroups) blocks = ngroups;
  if (blocks < 1) blocks = 1;
  switch (net.act) {
    case SPK_ACT_RELU:
      hipLaunchKernelGGL((ray_kernel<S, SPK_ACT_RELU>), dim3((unsigned)blocks), dim3(64), 0, stream, net, job);
      break;
    case SPK_ACT_ELU:
      hipLaunchKernelGGL((ray_kernel<S, SPK_ACT_ELU>), dim3((unsigned)blocks), dim3(64), 0, stream, net, job);
      break;
    default:
      hipLaunchKernelGGL((ray_kernel<S, SPK_ACT_SIN>), dim3((unsigned)blocks), dim3(64), 0, stream, net, job);
      break;
  }
  return hipGetLastError();
}

spk_status launch_rays(const spk_net* net, const spk_ray_params& p, int64_t n, const float* origin, const float* dir,
                       float* t_hit, int32_t* iters, unsigned long long* counter, hipStream_t stream, int num_cus) {
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
  if (hipGetLastError() != hipSuccess) return SPK_E_DEVICE;
  RayJob job;
  job.n = n;
  job.origin = origin;
  job.dir = dir;
  job.t_hit = t_hit;
  job.iters = iters;
  job.counter = counter;
  job.p = p;
  hipError_t e;
  switch (net->dev.H) {
    case 32: e = launch_rays_h<32>(net->dev, job, stream, num_cus); break;
    case 64: e = launch_rays_h<64>(net->dev, job, stream, num_cus); break;
    case 128: e = launch_rays_h<128>(net->dev, job, stream, num_cus); break;
    case 256: e = launch_rays_h<256>(net->dev, job, stream, num_cus); break;
    default: return SPK_E_UNSUPPORTED;
  }
  return e == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
