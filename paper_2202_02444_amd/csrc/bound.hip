// Batched range bound of an MLP over boxes (Procedure 1) on gfx950.
//
// See affine_core.h for the data layout.  Per wavefront and group of BPW
// boxes:
//   layer 0 (3 -> H)      VALU, owner layout (box -> affine form, Procedure 1
//                         step 1; Table 2 matrix multiplication)
//   activation + condense owner layout (eq. affine_func_update, Table 3,
//                         Section 3.3 fixed / truncate)
//   hidden layers         MFMA 16x16x4 FP32 for the generator columns Y = W X;
//                         the center column W x0 in FP64 and the products
//                         |W| xinf and |W| u (rounding-error column) on VALU
//                         alongside
//   output layer (H -> 1) VALU + segment reductions; range read-off
//                         (eq. def_range) and classification (Procedure 1).
//
// The center runs in FP64 because it carries the cancellation of every
// layer: in FP32 its rounding grows to ~1e-4 of the bound on 8-layer
// networks, while the generators and the condensed term stay accurate.
#include "affine_core.h"

namespace spk {

constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53

// Activation + condensation on the owner-layout rows.  On entry xc holds the
// pre-activation centers (FP64, bias included), y the generator terms in
// slots 1.. (slot 0 is unused), yinf the condensed term and e the error
// radius.  On exit xc/y/yinf/e hold the post-activation form and u = e + cK r
// + cD |x0| is the vector the next layer's rounding-error product |W| u needs.
// Returns the new number of occupied generator slots.
template <class S, int ACT, int POL>
__device__ __forceinline__ int activate(double (&xc)[4], float (&y)[4][S::NS], float (&yinf)[4], float (&e)[4],
                                        float (&u)[4], int n_occ, int k, float cK, float cD, float omega0, int lane,
                                        int16_t* rec) {
  float gam[4], rnext[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (ACT == SPK_ACT_SIN) {
      // Table 2 constant multiplication by omega0 before sin
      float rs = 0.0f;
#pragma unroll
      for (int C = 1; C < S::NS; ++C) {
        y[i][C] *= omega0;
        rs += fabsf(y[i][C]);
      }
      yinf[i] *= omega0;
      xc[i] *= (double)omega0;
      e[i] = (e[i] * omega0 + kU * (rs + yinf[i])) * kGrow + (float)(2.0 * kU64) * (float)fabs(xc[i]) + kEta;
    }
    const double x0 = xc[i];
    float rY = 0.0f;
#pragma unroll
    for (int C = 1; C < S::NS; ++C) rY += fabsf(y[i][C]);
    const float r = rY + yinf[i];
    const double xl = x0 - (double)r, xu = x0 + (double)r;
    const ActOut p = act_params<ACT>(xl, xu, x0);
    const float alf = (float)p.al;
    // rounding of the range read-off (the FP32 sum r)
    const float rho = (float)(S::NS + 3) * kU * r + kEta;
    const float ext = e[i] + rho;
    bool exact;
    if (ACT == SPK_ACT_RELU)
      exact = (p.al == 1.0 && xl - (double)ext >= 0.0) || (p.al == 0.0 && xu + (double)ext <= 0.0);
    else if (ACT == SPK_ACT_ELU)
      exact = p.al == 1.0 && xl - (double)ext >= 0.0;
    else
      exact = false;
    // the linearisation holds on [xl, xu] up to gamma; on the rounding
    // neighbourhood it degrades by at most lip * ext (unless it is exact there)
    float ep = fabsf(alf) * e[i] + (exact ? 0.0f : p.lip * ext + p.dg);
    const double z0 = fma(p.al, x0, p.be);
#pragma unroll
    for (int C = 1; C < S::NS; ++C) y[i][C] *= alf;
    xc[i] = z0;
    y[i][0] = (float)z0;
    const float zi = fabsf(alf) * yinf[i];
    // FP32 slope applied to the generators (2u: slope rounding + product),
    // condensed-term product, FP64 center update
    ep += 2.0f * kU * (fabsf(alf) * rY + zi) + (float)(2.0 * kU64) * (float)fabs(z0);
    yinf[i] = zi;
    // gamma rounded to FP32; the rounding goes into the error radius
    gam[i] = fmaxf((float)p.ga, 0.0f);
    e[i] = ep + kU * gam[i];
    rnext[i] = fabsf(alf) * r + gam[i];
  }

  int n_occ_new = n_occ;
  if (POL == SPK_AFFINE_FIXED) {
    // affine-fixed: every new term goes straight into the condensed coefficient
#pragma unroll
    for (int i = 0; i < 4; ++i) yinf[i] += gam[i];
  } else {
    // affine-truncate(k): candidates are the occupied old slots 1..n_occ
    // (magnitude = column L1 norm over the box's H rows) and the H new terms
    // (magnitude gamma_j); keep the k largest, ties to the lower candidate
    // index (old slots in slot order, then new terms by neuron index).
    constexpr int SEG = S::SEG;
    const int ch = lane % SEG;
    uint32_t kold[S::NS];
    kold[0] = 0u;
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const float mu = seg_allsum<SEG>((fabsf(y[0][C]) + fabsf(y[1][C])) + (fabsf(y[2][C]) + fabsf(y[3][C])));
      kold[C] = __float_as_uint(mu) & 0x7fffffffu;
    }
    uint32_t knew[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) knew[i] = __float_as_uint(gam[i]) & 0x7fffffffu;
    // old candidates this lane counts: slots C with (C-1) % SEG == ch
    constexpr int Q = (S::NS - 1 + SEG - 1) / SEG;
    uint32_t mine[Q];
    bool minev[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) { mine[q] = 0u; minev[q] = false; }
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const int q = (C - 1) / SEG;
      const bool sel = ((C - 1) % SEG) == ch;
      mine[q] = sel ? kold[C] : mine[q];
      minev[q] = sel ? (C <= n_occ) : minev[q];
    }
    // radix select of the k-th largest key, most significant bit first
    uint32_t T = 0u;
#pragma unroll 1
    for (int bit = 30; bit >= 0; --bit) {
      const uint32_t Tc = T | (1u << bit);
      int cnt = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) cnt += seg_count<SEG>(minev[q] && mine[q] >= Tc, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) cnt += seg_count<SEG>(knew[i] >= Tc, lane);
      T = (cnt >= k) ? Tc : T;
    }
    const uint32_t tau = T;
    int cgt = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) cgt += seg_count<SEG>(minev[q] && mine[q] > tau, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) cgt += seg_count<SEG>(knew[i] > tau, lane);
    const int need = k - cgt;
    // old slots: equal-to-tau ones ranked by slot
    uint32_t eqm = 0u, keep_old = 0u;
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const bool v = C <= n_occ;
      eqm |= (v && kold[C] == tau) ? (1u << C) : 0u;
    }
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      const bool v = C <= n_occ;
      const bool kp = v && (kold[C] > tau || (kold[C] == tau && __popc(eqm & ((1u << C) - 1u)) < need));
      keep_old |= kp ? (1u << C) : 0u;
    }
    const int n_eq_old = __popc(eqm);
    // new terms: rank among equal keys by neuron (row) index
    int run = n_eq_old;
#pragma unroll
    for (int i = 0; i < 4; ++i) run += seg_count_below<SEG>(knew[i] == tau, lane);
    bool keepnew[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool eq = knew[i] == tau;
      keepnew[i] = knew[i] > tau || (eq && run < need);
      run += eq ? 1 : 0;
    }
    // free slots (dropped old, then empty ones up to k) receive the kept new
    // terms in increasing slot order by increasing neuron index
    const uint32_t occm = (n_occ >= 31) ? 0xfffffffeu : ((1u << (n_occ + 1)) - 2u);
    const uint32_t kmsk = (k >= 31) ? 0xfffffffeu : ((1u << (k + 1)) - 2u);
    uint32_t freem = (occm & ~keep_old) | (kmsk & ~occm);
    if (S::BPW == 1) freem = __builtin_amdgcn_readfirstlane(freem);
    int rk = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) rk += seg_count_below<SEG>(keepnew[i], lane);
    int slot[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      slot[i] = keepnew[i] ? nth_set_bit(freem, rk) : -1;
      rk += keepnew[i] ? 1 : 0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float zi = yinf[i];
#pragma unroll
      for (int C = 1; C < S::NS; ++C) {
        if ((freem >> C) & 1u) {
          zi += fabsf(y[i][C]);
          y[i][C] = (slot[i] == C) ? gam[i] : 0.0f;
        }
      }
      zi += keepnew[i] ? 0.0f : gam[i];
      yinf[i] = zi;
    }
    if (rec != nullptr) {
      if (ch == 0) {
        for (int C = 0; C < 32; ++C) {
          const bool fr = (freem >> C) & 1u;
          if (!fr) rec[C] = (C == 0 || C <= k) ? (int16_t)-1 : (int16_t)-2;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (slot[i] >= 0) rec[slot[i]] = (int16_t)(4 * ch + i);
    }
    n_occ_new = (n_occ + S::H < k) ? n_occ + S::H : k;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float ef = e[i] * kGrow + (float)(S::NS + 2) * kU * yinf[i] + kEta;
    e[i] = ef;
    u[i] = ef + (cK * rnext[i] + cD * (float)fabs(xc[i])) * kGrowR;
  }
  return n_occ_new;
}

// Layer 0 in owner layout: affine form of the box (Procedure 1 step 1), then
// W0 x + b0.  Fills xc (FP64 centers), y (slots 1..s = box axes), yinf = 0
// and the error radius e.
template <class S>
__device__ __forceinline__ void layer0(const NetDev& net, const BoundJob& job, int64_t box, bool valid, int ch,
                                       double (&xc)[4], float (&y)[4][S::NS], float (&yinf)[4], float (&e)[4]) {
  double cc[3] = {0.0, 0.0, 0.0};
  float ax[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
  float ein[3] = {0.0f, 0.0f, 0.0f};
  if (valid) {
    if (job.mode == IN_GENERAL) {
#pragma unroll
      for (int d = 0; d < 3; ++d) cc[d] = (double)job.a[3 * box + d];
      for (int q = 0; q < job.s; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d) ax[q][d] = job.b[(box * job.s + q) * 3 + d];
    } else {
      float lo[3], hi[3];
      if (job.mode == IN_AABB) {
#pragma unroll
        for (int d = 0; d < 3; ++d) { lo[d] = job.a[3 * box + d]; hi[d] = job.b[3 * box + d]; }
      } else {
        // Morton cell at job.level: de-interleave the x, y, z indices
        const uint64_t code = job.cells[box];
        uint32_t idx[3] = {0u, 0u, 0u};
        for (int bb = 0; bb < job.level; ++bb) {
#pragma unroll
          for (int d = 0; d < 3; ++d) idx[d] |= (uint32_t)((code >> (3 * bb + d)) & 1ull) << bb;
        }
        const float scale = 1.0f / (float)(1u << job.level);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float size = (job.dom_hi[d] - job.dom_lo[d]) * scale;
          lo[d] = job.dom_lo[d] + (float)idx[d] * size;
          hi[d] = job.dom_lo[d] + (float)(idx[d] + 1u) * size;
        }
      }
      // center and half-width of the FP32 box, exactly, in FP64 (Procedure 3:
      // x_c = (x_l + x_u)/2, v = x_u - x_c); the half-width is then rounded to
      // FP32 for the generator, its rounding kept in ein
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        cc[d] = 0.5 * ((double)lo[d] + (double)hi[d]);
        const double h = (double)hi[d] - cc[d];
        ax[d][d] = (float)h;
        ein[d] = 2.0f * kU * fabsf((float)h) + kEta;
      }
    }
  }
  const f4* W0 = (const f4*)net.W0;   // rows padded to 4 floats
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = 4 * ch + i;
    const f4 w = W0[R];
    const float bb = net.b0[R];
    xc[i] = fma((double)w.z, cc[2], fma((double)w.y, cc[1], fma((double)w.x, cc[0], (double)bb)));
    const float cmag = (float)(fabs((double)w.x * cc[0]) + fabs((double)w.y * cc[1]) + fabs((double)w.z * cc[2])) +
                       fabsf(bb);
    float gmag = 0.0f;
    y[i][0] = (float)xc[i];
#pragma unroll
    for (int C = 1; C < S::NS; ++C) {
      if (C <= 3) {
        const int q = C - 1;
        const float v = fmaf(w.z, ax[q][2], fmaf(w.y, ax[q][1], w.x * ax[q][0]));
        y[i][C] = v;
        gmag += fabsf(w.x) * fabsf(ax[q][0]) + fabsf(w.y) * fabsf(ax[q][1]) + fabsf(w.z) * fabsf(ax[q][2]);
      } else {
        y[i][C] = 0.0f;
      }
    }
    yinf[i] = 0.0f;
    e[i] = (net.c3 * gmag + (float)(8.0 * kU64) * cmag + fabsf(w.x) * ein[0] + fabsf(w.y) * ein[1] +
            fabsf(w.z) * ein[2]) * kGrow + kEta;
  }
}

// Round a double to a float that is <= / >= it.
__device__ __forceinline__ float round_down_f(double v) {
  float f = (float)v;
  return ((double)f > v) ? next_down(f) : f;
}
__device__ __forceinline__ float round_up_f(double v) {
  float f = (float)v;
  return ((double)f < v) ? next_up(f) : f;
}

template <int SEG>
__device__ __forceinline__ double seg_allsum_d(double v) {
#pragma unroll
  for (int m = 1; m < SEG; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <class S, int ACT, int POL>
__global__ __launch_bounds__(64, 1) void bound_kernel(NetDev net, BoundJob job) {
  __shared__ __attribute__((aligned(16))) float tile[S::TILE];
  __shared__ __attribute__((aligned(16))) float vinf[256];
  __shared__ __attribute__((aligned(16))) float vu[256];
  __shared__ __attribute__((aligned(16))) double vc[256];

  constexpr int H = S::H, MT = S::MT, NT = S::NT, NS = S::NS, BPW = S::BPW, SEG = S::SEG;
  const int lane = threadIdx.x;
  const int g = lane >> 4, c = lane & 15;
  const int bo = lane / SEG;
  const int ch = lane % SEG;
  const int64_t ngroups = (job.n + BPW - 1) / BPW;
  const int L = net.L;
  const float cK = net.cK, cD = net.cD;
  const int k = job.k;

  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t box = grp * BPW + bo;
    const bool valid = box < job.n;
    double xc[4];
    float y[4][NS], yinf[4], e[4], u[4];
    layer0<S>(net, job, box, valid, ch, xc, y, yinf, e);
    int n_occ = job.s;
    for (int a = 0; a < L - 1; ++a) {
      int16_t* rec = nullptr;
      if (job.slot_src != nullptr && valid) rec = job.slot_src + ((size_t)a * job.n + box) * 32;
      n_occ = activate<S, ACT, POL>(xc, y, yinf, e, u, n_occ, k, cK, cD, net.omega0, lane, rec);
      if (a == L - 2) break;

      // ---- owner layout -> LDS ----
#pragma unroll
      for (int C = 0; C < NS; ++C) {
        f4 v = {y[0][C], y[1][C], y[2][C], y[3][C]};
        *(f4*)&tile[taddr<S>(bo, C, ch)] = v;
      }
      {
        f4 v1 = {yinf[0], yinf[1], yinf[2], yinf[3]};
        f4 v2 = {u[0], u[1], u[2], u[3]};
        *(f4*)&vinf[4 * lane] = v1;
        *(f4*)&vu[4 * lane] = v2;
#pragma unroll
        for (int i = 0; i < 4; ++i) vc[4 * lane + i] = xc[i];
      }
      __syncthreads();

      // ---- hidden layer a+1: generators on MFMA, center in FP64 ----
      f4 acc[MT][BPW * NT];
      float px[MT][BPW], pe[MT][BPW];
      double pd[MT][BPW];
#pragma unroll
      for (int tp = 0; tp < MT; ++tp) {
#pragma unroll
        for (int q = 0; q < BPW * NT; ++q) acc[tp][q] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < BPW; ++b) { px[tp][b] = 0.0f; pe[tp][b] = 0.0f; pd[tp][b] = 0.0; }
      }
      const f4* Wl = (const f4*)net.Wp + (size_t)a * (H * H / 4);
#pragma unroll 1
      for (int t = 0; t < MT; ++t) {
        f4 bfr[BPW][NT], vx[BPW], ve[BPW];
        double vd[BPW][4];
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
#pragma unroll
          for (int n = 0; n < NT; ++n) bfr[b][n] = *(const f4*)&tile[taddr<S>(b, 16 * n + c, 4 * t + g)];
          vx[b] = *(const f4*)&vinf[b * H + 16 * t + 4 * g];
          ve[b] = *(const f4*)&vu[b * H + 16 * t + 4 * g];
#pragma unroll
          for (int j = 0; j < 4; ++j) vd[b][j] = vc[b * H + 16 * t + 4 * g + j];
        }
        const f4* Wt = Wl + (size_t)t * MT * 64 + lane;
#pragma unroll
        for (int tp = 0; tp < MT; ++tp) {
          const f4 w = Wt[tp * 64];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double wd = (double)w[j];
#pragma unroll
            for (int b = 0; b < BPW; ++b) {
#pragma unroll
              for (int n = 0; n < NT; ++n)
                acc[tp][b * NT + n] =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(w[j], bfr[b][n][j], acc[tp][b * NT + n], 0, 0, 0);
              px[tp][b] = fmaf(fabsf(w[j]), vx[b][j], px[tp][b]);
              pe[tp][b] = fmaf(fabsf(w[j]), ve[b][j], pe[tp][b]);
              pd[tp][b] = fma(wd, vd[b][j], pd[tp][b]);
            }
          }
        }
      }
      __syncthreads();

      // ---- MFMA layout -> LDS -> owner layout ----
#pragma unroll
      for (int tp = 0; tp < MT; ++tp) {
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
          float sx = px[tp][b], se = pe[tp][b];
          double sd = pd[tp][b];
          sx += __shfl_xor(sx, 16, 64);
          se += __shfl_xor(se, 16, 64);
          sd += __shfl_xor(sd, 16, 64);
          sx += __shfl_xor(sx, 32, 64);
          se += __shfl_xor(se, 32, 64);
          sd += __shfl_xor(sd, 32, 64);
          if (g == 0) {
            vinf[b * H + 16 * tp + c] = sx;
            vu[b * H + 16 * tp + c] = se;
            vc[b * H + 16 * tp + c] = sd;
          }
#pragma unroll
          for (int n = 0; n < NT; ++n) *(f4*)&tile[taddr<S>(b, 16 * n + c, 4 * tp + g)] = acc[tp][b * NT + n];
        }
      }
      __syncthreads();
#pragma unroll
      for (int C = 1; C < NS; ++C) {
        const f4 v = *(const f4*)&tile[taddr<S>(bo, C, ch)];
        y[0][C] = v.x; y[1][C] = v.y; y[2][C] = v.z; y[3][C] = v.w;
      }
      {
        const f4 xi = *(const f4*)&vinf[4 * lane];
        const f4 eu = *(const f4*)&vu[4 * lane];
        const f4 bh = *(const f4*)&net.bh[(size_t)a * H + 4 * ch];
        const f4 eb = *(const f4*)&net.ebh[(size_t)a * H + 4 * ch];
        const float grow = 1.0f + 2.0f * cK;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          xc[i] = vc[4 * lane + i] + (double)bh[i];
          y[i][0] = (float)xc[i];
          yinf[i] = xi[i];
          e[i] = eu[i] * grow + eb[i];
        }
      }
      __syncthreads();
    }

    // ---- output layer (H -> 1) and range read-off ----
    const f4 wv = *(const f4*)&net.wL[4 * ch];
    double p0 = 0.0;
    float pinf = 0.0f, pu = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      p0 = fma((double)wv[i], xc[i], p0);
      pinf = fmaf(fabsf(wv[i]), yinf[i], pinf);
      pu = fmaf(fabsf(wv[i]), u[i], pu);
    }
    p0 = seg_allsum_d<SEG>(p0);
    pinf = seg_allsum<SEG>(pinf);
    pu = seg_allsum<SEG>(pu);
    float r = 0.0f;
#pragma unroll
    for (int C = 1; C < NS; ++C) {
      float pc = wv[0] * y[0][C];
      pc = fmaf(wv[1], y[1][C], pc);
      pc = fmaf(wv[2], y[2][C], pc);
      pc = fmaf(wv[3], y[3][C], pc);
      r += fabsf(seg_allsum<SEG>(pc));
    }
    r += pinf;
    const double y0 = p0 + (double)net.bL;
    const float err = (pu * (1.0f + 2.0f * cK) + net.eL + (float)(NS + 3) * kU * r +
                       (float)(4.0 * kU64) * (float)fabs(y0)) * kGrow + kEta;
    if (valid && ch == 0) {
      const double s = ((double)r + (double)err) * (1.0 + 4.0 * kU64);
      float lo = round_down_f(y0 - s);
      float hi = round_up_f(y0 + s);
      if (!(lo <= hi) || !(lo > -INFINITY) || !(hi < INFINITY)) {
        lo = -INFINITY;
        hi = INFINITY;
      }
      if (job.lo) job.lo[box] = lo;
      if (job.hi) job.hi[box] = hi;
      if (job.label) job.label[box] = (lo > 0.0f) ? (uint8_t)SPK_POSITIVE
                                      : (hi < 0.0f) ? (uint8_t)SPK_NEGATIVE : (uint8_t)SPK_UNKNOWN;
      if (job.center) job.center[box] = (float)y0;
      if (job.radius) job.radius[box] = r;
      if (job.err) job.err[box] = err;
    }
  }
}

template <class S, int ACT, int POL>
static hipError_t launch_one(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  const int64_t ngroups = (job.n + S::BPW - 1) / S::BPW;
  int64_t blocks = (int64_t)num_cus * 4;
  if (blocks > ngroups) blocks = ngroups;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((bound_kernel<S, ACT, POL>), dim3((unsigned)blocks), dim3(64), 0, stream, net, job);
  return hipGetLastError();
}

template <int H, int NT, int POL>
static hipError_t launch_act(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  switch (net.act) {
    case SPK_ACT_RELU: return launch_one<Shape<H, NT>, SPK_ACT_RELU, POL>(net, job, stream, num_cus);
    case SPK_ACT_ELU: return launch_one<Shape<H, NT>, SPK_ACT_ELU, POL>(net, job, stream, num_cus);
    case SPK_ACT_SIN: return launch_one<Shape<H, NT>, SPK_ACT_SIN, POL>(net, job, stream, num_cus);
  }
  return hipErrorInvalidValue;
}

template <int H>
static hipError_t launch_h(const NetDev& net, const BoundJob& job, hipStream_t stream, int num_cus) {
  if (job.policy == SPK_AFFINE_FIXED) return launch_act<H, 1, SPK_AFFINE_FIXED>(net, job, stream, num_cus);
  if (job.k <= 15) return launch_act<H, 1, SPK_AFFINE_TRUNCATE>(net, job, stream, num_cus);
  return launch_act<H, 2, SPK_AFFINE_TRUNCATE>(net, job, stream, num_cus);
}

spk_status launch_bound(const spk_net* net, const BoundJob& job, hipStream_t stream, int num_cus) {
  if (job.n <= 0) return SPK_OK;
  hipError_t err;
  switch (net->dev.H) {
    case 32: err = launch_h<32>(net->dev, job, stream, num_cus); break;
    case 64: err = launch_h<64>(net->dev, job, stream, num_cus); break;
    case 128: err = launch_h<128>(net->dev, job, stream, num_cus); break;
    case 256: err = launch_h<256>(net->dev, job, stream, num_cus); break;
    default: return SPK_E_UNSUPPORTED;
  }
  return err == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

}  // namespace spk
