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
//
// By default the segment bounds carry the rounding bound of every layer (the
// same folding as the box bounds), so a step is accepted only when the exact
// network has no root on the segment; SPK_FLAG_NO_ROUNDING_BOUND selects the
// paper's arithmetic with the tolerance margin.
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
  const bool rig = (P.flags & SPK_FLAG_NO_ROUNDING_BOUND) == 0;

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
    float yinf[4], e[4], u[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    layer0_affine<S, NPASS>(net, ch, cc, ax, ein, pts, xc, y, yinf, e);
    for (int a = 0; a < L - 1; ++a) {
      activate<S, ACT, SPK_AFFINE_FIXED, NPASS>(xc, y, yinf, e, u, 1, 0, net.cK, net.cD, net.omega0, lane,
                                                  nullptr, nullptr, rig);
      if (a == L - 2) break;
      hidden_layer<S, NPASS>(net, sm, a, xc, y, yinf, e, u, lane, rig);
    }
    float pass[NPASS];
    const OutVals o = output_layer<S, NPASS>(net, xc, y, yinf, u, lane, pass, rig);

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
        enclose(o, rig, lo, hi);
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

// ---------------------------------------------------------------------------
// Packed ray marching for hidden width 256: one wavefront marches RPW rays
// at once.  Each ray takes three term slots of one 16-slot tile (its segment
// generator and its two passenger points), so one MFMA pass serves RPW rays.
// The FP64 centers and |W| xinf of the RPW rays are row-owner dot products
// (lane l owns rows 4l..4l+3) over a copy of W in 4x4 blocks (one coalesced
// 4 KB load per wave and k step), sharing each weight conversion across the
// rays.  Ray state is uniform across the wavefront.
// ---------------------------------------------------------------------------
constexpr int RPW = 5;

template <class S>
struct PackedRayLds {
  LdsState<S> base;              // the 16-slot tile
  float vinf[RPW][256];
  double vc[RPW][256];
};

__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni(long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(unsigned long long)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Activation (affine-fixed) of every ray's rows; passengers get f exactly.
// With rig the rounding errors are folded into yinf as in activate(): the
// errors of the producing layer are already in yinf (added where they arise,
// so no separate register array is live), the linearisation is taken on the
// whole range, the rounding of the update follows, then the a-priori rounding
// of the next layer's products (cK |y| + cD |x0|).
template <int ACT>
__device__ __forceinline__ void activate_packed(double (&xc)[RPW][4], f4 (&y)[16], float (&yinf)[RPW][4],
                                                const NetDev& net, bool rig) {
  const float omega0 = net.omega0;
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int G = 1 + 3 * r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      y[G + 1][i] = act_point<ACT>(y[G + 1][i], omega0);
      y[G + 2][i] = act_point<ACT>(y[G + 2][i], omega0);
      if (ACT == SPK_ACT_SIN) {
        y[G][i] *= omega0;
        xc[r][i] *= (double)omega0;
        if (rig) {
          const double ys = (double)yinf[r][i] * (double)omega0;
          yinf[r][i] = round_up_f((ys + (double)kU * ((double)fabsf(y[G][i]) + ys)) * (1.0 + 4.0 * kU64) +
                                  2.0 * kU64 * fabs(xc[r][i]) + (double)kEta);
        } else {
          yinf[r][i] *= omega0;
        }
      }
      const double x0 = xc[r][i];
      const float rY = fabsf(y[G][i]);
      double rd = (double)rY + (double)yinf[r][i];
      if (rig) rd = rd * (1.0 + 4.0 * kU64) + (double)kEta;
      const ActOut p = act_params<ACT>(x0 - rd, x0 + rd, x0);
      const float alf = (float)p.al;
      y[G][i] *= alf;
      const double z0 = fma(p.al, x0, p.be);
      xc[r][i] = z0;
      const float zi = fabsf(alf) * yinf[r][i];
      const float gam = fmaxf((float)p.ga, 0.0f);
      if (rig) {
        const double ep = 2.0 * (double)kU * ((double)fabsf(alf) * (double)rY + (double)zi) + 2.0 * kU64 * fabs(z0) +
                          (double)kU * (double)gam + (double)p.dg + (double)kEta;
        const double zf = ((double)zi + ep + (double)gam) * (1.0 + 4.0 * kU64);
        const double rnext = (double)fabsf(alf) * (double)round_up_f(rd) + (double)gam;
        yinf[r][i] = round_up_f((double)round_up_f(zf) +
                                ((double)net.cK * rnext + (double)net.cD * fabs(z0)) * (1.0 + 1.52587890625e-05) +
                                (double)kEta);
      } else {
        yinf[r][i] = zi + gam;
      }
    }
  }
}

// Generator columns of the tile on MFMA (16x16x4 FP32, one K block of 16 per
// step) with the row-owner products of every ray interleaved: one k step of
// 4 per four row tiles, its weights loaded at the first of them and its rays
// spread over the other three (2 + 2 + 1 rays), so that every group of four
// MFMAs has VALU work beside it.
template <class S>
__device__ __forceinline__ void packed_pass(PackedRayLds<S>& sm, const f4* Wl, const f4* Wr0, int lane,
                                            double (&pd)[RPW][4], float (&px)[RPW][4]) {
  constexpr int MT = S::MT, PF = 4, H = S::H;
  static_assert(MT % 4 == 0 && MT % PF == 0, "four row tiles per k step");
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      pd[r][i] = 0.0;
      px[r][i] = 0.0f;
    }
  f4 acc[MT];
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) acc[tp] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
  const f4* Wq = Wl + lane;
  const f4* Wr = Wr0 + 4 * lane;
  f4 ring[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) ring[p] = Wq[p * 64];
  f4 bn = *(const f4*)&sm.base.tile[taddr<S>(0, c, g)];
#pragma unroll 1
  for (int t = 0; t < MT; ++t) {
    const f4 bfr = bn;
    const int t1 = min(t + 1, MT - 1);
    bn = *(const f4*)&sm.base.tile[taddr<S>(0, c, 4 * t1 + g)];
    f4 wv[4];
    double wd[4][4];
#pragma unroll
    for (int tp = 0; tp < MT; ++tp) {
      const int k = 16 * t + 4 * (tp >> 2);
      if ((tp & 3) == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) wv[i] = Wr[(size_t)(k / 4) * H + i];
      }
      const f4 w = ring[tp % PF];
      const int qn = min(t * MT + tp + PF, MT * MT - 1);   // past the end: a harmless reload
      ring[tp % PF] = Wq[(size_t)qn * 64];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[tp] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[j], bfr[j], acc[tp], 0, 0, 0);
      if ((tp & 3) >= 1) {
        if ((tp & 3) == 1) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) wd[i][j] = (double)wv[i][j];
        }
        const int rb = (tp & 3) == 1 ? 0 : ((tp & 3) == 2 ? 2 : 4);
        const int re = (tp & 3) == 3 ? RPW : rb + 2;
#pragma unroll
        for (int r = rb; r < re; ++r) {
          const f4 xi = *(const f4*)&sm.vinf[r][k];
          double xd[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) xd[j] = sm.vc[r][k + j];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              pd[r][i] = fma(wd[i][j], xd[j], pd[r][i]);
              px[r][i] = fmaf(fabsf(wv[i][j]), xi[j], px[r][i]);
            }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int tp = 0; tp < MT; ++tp) *(f4*)&sm.base.tile[taddr<S>(0, c, 4 * tp + g)] = acc[tp];
  __syncthreads();
}

// One H -> H layer for the packed rays.
template <class S>
__device__ __forceinline__ void hidden_packed(const NetDev& net, PackedRayLds<S>& sm, int a, double (&xc)[RPW][4],
                                              f4 (&y)[16], float (&yinf)[RPW][4], int lane, bool rig) {
  constexpr int H = S::H;
#pragma unroll
  for (int C = 0; C < 16; ++C) *(f4*)&sm.base.tile[taddr<S>(0, C, lane)] = y[C];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    *(f4*)&sm.vinf[r][4 * lane] = (f4){yinf[r][0], yinf[r][1], yinf[r][2], yinf[r][3]};
#pragma unroll
    for (int i = 0; i < 4; ++i) sm.vc[r][4 * lane + i] = xc[r][i];
  }
  __syncthreads();
  double pd[RPW][4];
  float px[RPW][4];
  packed_pass<S>(sm, (const f4*)net.Wp + (size_t)a * (H * H / 4), (const f4*)(net.Wr + (size_t)a * H * H), lane,
                 pd, px);
#pragma unroll
  for (int C = 1; C < 16; ++C) y[C] = *(const f4*)&sm.base.tile[taddr<S>(0, C, lane)];
  const f4 bh = *(const f4*)&net.bh[(size_t)a * H + 4 * lane];
  const f4 eb = *(const f4*)&net.ebh[(size_t)a * H + 4 * lane];
  const double grow = 1.0 + 2.0 * (double)net.cK;
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int G = 1 + 3 * r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xc[r][i] = pd[r][i] + (double)bh[i];
      // rigorous: |W| yinf summed in FP32 (rounded up by its a-priori bound),
      // the bias terms and the bias addition of the FP64 center
      yinf[r][i] = rig ? round_up_f(((double)px[r][i] * grow + (double)eb[i] + 2.0 * kU64 * fabs(xc[r][i])) *
                                    (1.0 + 2.0 * kU64))
                       : px[r][i];
      y[G + 1][i] += bh[i];
      y[G + 2][i] += bh[i];
    }
  }
  __syncthreads();
}

template <class S, int ACT, bool RIG>
__global__ __launch_bounds__(64, 1) void ray_kernel_packed(NetDev net, RayJob job) {
  static_assert(S::H == 256 && S::NT == 1, "packed rays: width 256, one 16-slot tile");
  __shared__ __attribute__((aligned(16))) PackedRayLds<S> sm;
  const int lane = threadIdx.x;
  const int L = net.L;
  const spk_ray_params P = job.p;
  // a template flag: both variants stay free of scratch spills
  constexpr bool rig = RIG;

  long long rid[RPW];
  float t[RPW], sigma[RPW], f0[RPW], tmax[RPW], base[RPW], sp[RPW][3], dv[RPW][3];
  int it[RPW], first[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    rid[r] = -1;
    t[r] = sigma[r] = f0[r] = tmax[r] = base[r] = 0.0f;
    it[r] = first[r] = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) sp[r][a] = dv[r][a] = 0.0f;
  }

  for (;;) {
    // ---- refill empty slots from the global counter (lane 0), broadcast
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      if (rid[r] != -1) continue;   // uniform
      long long nr = -2;
      float np[3] = {0.0f, 0.0f, 0.0f}, nd[3] = {0.0f, 0.0f, 0.0f}, ntmax = 0.0f, nbase = 0.0f;
      if (lane == 0) {
        for (;;) {
          const unsigned long long idx = atomicAdd(job.counter, 1ull);
          if (idx >= (unsigned long long)job.n) break;
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
      nr = uni(nr);
      if (nr >= 0) {
        rid[r] = nr;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          sp[r][a] = uni(np[a]);
          dv[r][a] = uni(nd[a]);
        }
        tmax[r] = uni(ntmax);
        base[r] = uni(nbase);
        t[r] = 0.0f;
        sigma[r] = P.sigma0;
        it[r] = 0;
        first[r] = 1;
      } else {
        rid[r] = -2;
      }
    }
    bool any = false;
#pragma unroll
    for (int r = 0; r < RPW; ++r) any = any || rid[r] >= 0;
    if (!any) break;   // uniform: every slot drained and no rays left

    // ---- layer 0 for every ray: segment [t, t + sigma] and two passenger points
    double xc[RPW][4];
    f4 y[16];
    float yinf[RPW][4];
    {
      const f4* W0 = (const f4*)net.W0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int R = 4 * lane + i;
        const f4 w = W0[R];
        const float bb = net.b0[R];
        y[0][i] = 0.0f;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const int G = 1 + 3 * r;
          const bool act = rid[r] >= 0;
          double cc[3];
          float ax[3], p0[3], p1[3], ein[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            cc[a] = act ? (double)sp[r][a] + ((double)t[r] + 0.5 * (double)sigma[r]) * (double)dv[r][a] : 0.0;
            const double v = act ? 0.5 * (double)sigma[r] * (double)dv[r][a] : 0.0;
            ax[a] = (float)v;
            // the segment's center and half-axis as computed against the exact
            // segment of the ray (FP64 center, FP32 axis)
            ein[a] = 2.0f * kU * fabsf((float)v) + (float)(4.0 * kU64) * (float)fabs(cc[a]) + kEta;
            p0[a] = act ? sp[r][a] + (t[r] + P.delta) * dv[r][a] : 0.0f;
            p1[a] = act ? sp[r][a] : 0.0f;
          }
          xc[r][i] = fma((double)w.z, cc[2], fma((double)w.y, cc[1], fma((double)w.x, cc[0], (double)bb)));
          y[G][i] = fmaf(w.z, ax[2], fmaf(w.y, ax[1], w.x * ax[0]));
          y[G + 1][i] = fmaf(w.z, p0[2], fmaf(w.y, p0[1], fmaf(w.x, p0[0], bb)));
          y[G + 2][i] = fmaf(w.z, p1[2], fmaf(w.y, p1[1], fmaf(w.x, p1[0], bb)));
          // rigorous: FP32 three-term generator product, FP64 center, input error
          const float gmag = fabsf(w.x) * fabsf(ax[0]) + fabsf(w.y) * fabsf(ax[1]) + fabsf(w.z) * fabsf(ax[2]);
          const float cmag = (float)(fabs((double)w.x * cc[0]) + fabs((double)w.y * cc[1]) +
                                     fabs((double)w.z * cc[2])) + fabsf(bb);
          yinf[r][i] = rig ? (net.c3 * gmag + (float)(8.0 * kU64) * cmag + fabsf(w.x) * ein[0] +
                              fabsf(w.y) * ein[1] + fabsf(w.z) * ein[2]) * kGrow + kEta
                           : 0.0f;
        }
      }
    }
    for (int a = 0; a < L - 1; ++a) {
      activate_packed<ACT>(xc, y, yinf, net, rig);
      if (a == L - 2) break;
      hidden_packed<S>(net, sm, a, xc, y, yinf, lane, rig);
    }
    // ---- output layer per ray and the Procedure 2 update (uniform)
    const f4 wv = *(const f4*)&net.wL[4 * lane];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int G = 1 + 3 * r;
      double p0 = 0.0;
      float pinf = 0.0f, pg = 0.0f, q0 = 0.0f, q1 = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        p0 = fma((double)wv[i], xc[r][i], p0);
        pinf = fmaf(fabsf(wv[i]), yinf[r][i], pinf);
        pg = fmaf(wv[i], y[G][i], pg);
        q0 = fmaf(wv[i], y[G + 1][i], q0);
        q1 = fmaf(wv[i], y[G + 2][i], q1);
      }
      p0 = seg_allsum_d<64>(p0);
      pinf = seg_allsum<64>(pinf);
      pg = seg_allsum<64>(pg);
      q0 = seg_allsum<64>(q0) + net.bL;
      q1 = seg_allsum<64>(q1) + net.bL;
      if (rid[r] < 0) continue;
      OutVals o;
      o.y0 = p0 + (double)net.bL;
      if (rig) {
        // the products' rounding is already in yinf (folded by the last
        // activation); add the rounding of |w| yinf, the output bias and the
        // center
        o.r = round_up_f(((double)fabsf(pg) + (double)pinf) * (1.0 + 4.0 * kU64));
        o.err = round_up_f((2.0 * (double)net.cK * (double)pinf + (double)net.eL + 4.0 * kU64 * fabs(o.y0)) *
                               (1.0 + 4.0 * kU64) + (double)kEta);
      } else {
        o.r = (float)((double)fabsf(pg) + (double)pinf);
        o.err = 0.0f;
      }
      if (first[r]) {
        f0[r] = q1;
        first[r] = 0;
      }
      ++it[r];
      if ((f0[r] > 0.0f) != (q0 > 0.0f)) {
        if (lane == 0) {
          job.t_hit[rid[r]] = base[r] + t[r];
          if (job.iters) job.iters[rid[r]] = it[r];
        }
        rid[r] = -1;
      } else {
        float lo, hi;
        enclose(o, rig, lo, hi);
        const bool safe = lo > 0.0f || hi < 0.0f;
        const float step = safe ? P.safety * sigma[r] : 0.0f;
        sigma[r] = safe ? sigma[r] * P.eta_plus : sigma[r] * P.eta_minus;
        t[r] += fmaxf(step, P.delta);
        if (!(t[r] < tmax[r]) || it[r] >= P.max_iters) {
          if (lane == 0) {
            job.t_hit[rid[r]] = INFINITY;
            if (job.iters) job.iters[rid[r]] = it[r];
          }
          rid[r] = -1;
        }
      }
    }
  }
}

template <int H>
static hipError_t launch_rays_h(const NetDev& net, const RayJob& job, hipStream_t stream, int num_cus) {
  using S = Shape<H, 1>;
  if constexpr (H == 256) {
    const int64_t nw = (job.n + RPW - 1) / RPW;
    int64_t blocks = (int64_t)num_cus * 4;
    if (blocks > nw) blocks = nw;
    if (blocks < 1) blocks = 1;
    const bool rig = (job.p.flags & SPK_FLAG_NO_ROUNDING_BOUND) == 0;
    switch (net.act) {
      case SPK_ACT_RELU:
        if (rig)
          hipLaunchKernelGGL((ray_kernel_packed<S, SPK_ACT_RELU, true>), dim3((unsigned)blocks), dim3(64), 0, stream,
                             net, job);
        else
          hipLaunchKernelGGL((ray_kernel_packed<S, SPK_ACT_RELU, false>), dim3((unsigned)blocks), dim3(64), 0, stream,
                             net, job);
        break;
      case SPK_ACT_ELU:
        if (rig)
          hipLaunchKernelGGL((ray_kernel_packed<S, SPK_ACT_ELU, true>), dim3((unsigned)blocks), dim3(64), 0, stream,
                             net, job);
        else
          hipLaunchKernelGGL((ray_kernel_packed<S, SPK_ACT_ELU, false>), dim3((unsigned)blocks), dim3(64), 0, stream,
                             net, job);
        break;
      default:
        if (rig)
          hipLaunchKernelGGL((ray_kernel_packed<S, SPK_ACT_SIN, true>), dim3((unsigned)blocks), dim3(64), 0, stream,
                             net, job);
        else
          hipLaunchKernelGGL((ray_kernel_packed<S, SPK_ACT_SIN, false>), dim3((unsigned)blocks), dim3(64), 0, stream,
                             net, job);
        break;
    }
    return hipGetLastError();
  }
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
