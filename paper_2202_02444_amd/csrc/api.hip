// C ABI of the library: argument validation, the device network store and
// the launch sequence of every entry point.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "spk_impl.h"

using namespace spk;

namespace {

// Round a non-negative double up to a float that is >= it.
float up_f32(double v) {
  float f = (float)v;
  if ((double)f < v) f = nextafterf(f, INFINITY);
  return f;
}

// Relative rounding constant of an n-term FP32 dot product plus a bias term,
// with every multiply and add faithfully rounded (error <= 2^-23 relative),
// in any accumulation order: gamma = m u' / (1 - m u'), m = n + 2, u' = 2^-23.
double dot_const(int n, int mantissa_bits) {
  const double up = ldexp(1.0, -(mantissa_bits - 1));
  const double m = (double)n + 2.0;
  return m * up / (1.0 - m * up) * (1.0 + 1e-6);
}

// Round-to-nearest-even BF16 (the upper 16 bits of an FP32) of a finite float.
uint16_t bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// Relative error bound of a split-BF16 H-term dot product (hi/lo parts of
// both operands, the three cross products hi*hi + hi*lo + lo*hi accumulated
// in FP32), against sum |w||x|: each operand is w = hi + lo + dw with
// |lo| <= u_b (1 + u_b) |w| and |dw| <= u_b^2 |w| (u_b = 2^-8, round to
// nearest), so the dropped lo*lo and the residual terms stay below
// 3 u_b^2 (1 + 2 u_b) |w||x|; the 3H exact products are then summed in FP32,
// their magnitudes |hi||hi| + |hi||lo| + |lo||hi| below (1 + 2^-7) |w||x|.
double split_const(int H) {
  const double ub = ldexp(1.0, -8);
  return 3.0 * ub * ub * (1.0 + 2.0 * ub) * (1.0 + 1e-6) + dot_const(3 * H, 24) * (1.0 + ldexp(1.0, -7));
}

// Binary16 of a finite double with |v| < 65520: round to nearest even on an
// 11-bit significand; results below the smallest normal (2^-14) are stored as
// zero, so no FP16 subnormal ever reaches the MFMA.  *val receives the value.
uint16_t f16_rne_ftz(double v, double* val) {
  const double a = fabs(v);
  const uint16_t sign = std::signbit(v) ? 0x8000u : 0u;
  *val = 0.0;
  if (a == 0.0) return sign;
  int e = 0;
  (void)frexp(a, &e);                          // a in [2^(e-1), 2^e)
  const double q = ldexp(1.0, e - 11);         // quantum of an 11-bit significand
  const double r = rint(a / q) * q;            // ties to even (default rounding mode)
  if (r < ldexp(1.0, -14)) return sign;
  int e2 = 0;
  (void)frexp(r, &e2);
  const int E = e2 - 1;                        // r in [2^E, 2^(E+1))
  const uint16_t mant = (uint16_t)(ldexp(r, -E) * 1024.0 - 1024.0);
  *val = std::signbit(v) ? -r : r;
  return (uint16_t)(sign | (uint16_t)((E + 15) << 10) | mant);
}

// Relative error bound of a scaled split-FP16 H-term dot product against
// sum |w'||x'| (scaled operands v' = hi + lo + dv, hi = RNE16(v'),
// lo = RNE16(v' - hi)): the dropped lo*lo term (<= 2^-22 (1 + 2^-11)^2), the
// X residual (<= 2^-22 |x'| (1 + 2^-11) plus an absolute part accounted per
// column), the relative W residual cw (measured exactly over the stored
// split; weights with a subnormal lo part are accounted absolutely per row),
// and FP32 accumulation of the 3H exact products.
double split16_const(int H, double cw) {
  const double u11 = ldexp(1.0, -11), u22 = ldexp(1.0, -22);
  // |W_hi + W_lo| <= (1 + 2^-10) |W'| for every weight (cw <= 2^-21; the
  // absolutely accounted ones have |dw| <= 2^-11 |W'|); the accumulated
  // magnitudes sum |hi||hi| + |hi||lo| + |lo||hi| stay below (1 + 2^-9) sum |w'||x'|
  const double rel = u22 * (1.0 + u11) * (1.0 + u11) + u22 * (1.0 + u11) * (1.0 + 2.0 * u11) + cw;
  return rel * (1.0 + 1e-6) + dot_const(3 * H, 24) * (1.0 + ldexp(1.0, -9));
}

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(p[i])) return false;
  return true;
}

spk_status check_hip(hipError_t e) { return e == hipSuccess ? SPK_OK : SPK_E_DEVICE; }


}  // namespace

// Fixed scratch of spk_subdivide_frontier_noalloc: the per-cell labels of one
// frontier round (one byte per cell).  Every GPU the library runs on holds its
// own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for that device (the array's name is not
// a device address on the host).
static __device__ __align__(256) uint8_t scratch[SPK_NOALLOC_MAX_CELLS];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with that
// device current (the caller's current device is restored).
static spk_status noalloc_scratch(int device, void** p) {
  if (device < 0 || device >= kMaxDevices) return SPK_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return SPK_E_DEVICE;
    if (cur != device && hipSetDevice(device) != hipSuccess) return SPK_E_DEVICE;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || ptr == nullptr) return SPK_E_DEVICE;
    g_scratch_ptr[device] = ptr;
  }
  *p = g_scratch_ptr[device];
  return SPK_OK;
}

namespace spk {
void net_mark_use(const spk_net* net, hipStream_t stream) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lock(net->use_mu);
  hipEvent_t ev = nullptr;
  for (auto& u : net->uses)
    if (u.first == stream) ev = u.second;
  if (ev == nullptr) {
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return;
    net->uses.emplace_back(stream, ev);
  }
  (void)hipEventRecord(ev, stream);
}
}  // namespace spk

extern "C" {

const char* spk_status_str(spk_status s) {
  switch (s) {
    case SPK_OK: return "ok";
    case SPK_E_INVAL: return "invalid argument";
    case SPK_E_NOMEM: return "out of memory";
    case SPK_E_NOSPC: return "output capacity too small";
    case SPK_E_DEVICE: return "HIP runtime error";
    case SPK_E_UNSUPPORTED: return "not supported by the library";
    case SPK_E_BUSY: return "object busy";
    case SPK_E_LIMIT: return "request exceeds a fixed capacity of the library";
  }
  return "unknown status";
}

const char* spk_version(void) { return "spk 0.1 gfx950"; }

spk_status spk_net_create(int32_t n_linear, const int32_t* widths, const float* const* W, const float* const* b,
                          int32_t act, float omega0, spk_net** out) {
  if (out == nullptr || widths == nullptr || W == nullptr || b == nullptr) return SPK_E_INVAL;
  *out = nullptr;
  if (n_linear < 2 || n_linear > 16) return SPK_E_UNSUPPORTED;
  if (act != SPK_ACT_RELU && act != SPK_ACT_ELU && act != SPK_ACT_SIN) return SPK_E_INVAL;
  if (act == SPK_ACT_SIN && !(omega0 > 0.0f && isfinite(omega0))) return SPK_E_INVAL;
  if (widths[0] != 3 || widths[n_linear] != 1) return SPK_E_UNSUPPORTED;
  const int H = widths[1];
  if (H != 32 && H != 64 && H != 128 && H != 256) return SPK_E_UNSUPPORTED;
  for (int l = 1; l < n_linear; ++l)
    if (widths[l] != H) return SPK_E_UNSUPPORTED;
  for (int l = 0; l < n_linear; ++l) {
    if (W[l] == nullptr || b[l] == nullptr) return SPK_E_INVAL;
    if (!finite_all(W[l], (size_t)widths[l] * widths[l + 1]) || !finite_all(b[l], (size_t)widths[l + 1]))
      return SPK_E_INVAL;
  }
  const int L = n_linear;
  const double cK = dot_const(H, 24);
  const double cD = dot_const(H, 53);
  const double c3 = dot_const(3, 24);
  const double eta = ldexp(1.0, -100);

  // host images of every device array
  const size_t nW0 = (size_t)H * 4, nb0 = H, nWp = (size_t)(L - 2) * H * H, nbh = (size_t)(L - 2) * H;
  std::vector<float> W0(nW0, 0.0f), b0(nb0), Wp(nWp), bh(nbh), ebh(nbh), wL(H);
  for (int r = 0; r < H; ++r) {
    for (int d = 0; d < 3; ++d) W0[(size_t)r * 4 + d] = W[0][(size_t)r * 3 + d];
    b0[r] = b[0][r];
  }
  const int MT = H / 16;
  for (int l = 1; l <= L - 2; ++l) {
    const float* Wl = W[l];
    float* dst = Wp.data() + (size_t)(l - 1) * H * H;
    // A-fragment order: [t][tp][lane][j] = W[16 tp + c][16 t + 4 g + j], lane = 16 g + c
    for (int t = 0; t < MT; ++t)
      for (int tp = 0; tp < MT; ++tp)
        for (int lane = 0; lane < 64; ++lane)
          for (int j = 0; j < 4; ++j) {
            const int g = lane >> 4, c = lane & 15;
            const int row = 16 * tp + c, col = 16 * t + 4 * g + j;
            dst[(((size_t)t * MT + tp) * 64 + lane) * 4 + j] = Wl[(size_t)row * H + col];
          }
    for (int r = 0; r < H; ++r) {
      const float bv = b[l][r];
      bh[(size_t)(l - 1) * H + r] = bv;
      ebh[(size_t)(l - 1) * H + r] = up_f32(cK * fabs((double)bv) + eta);
    }
  }
  // split-BF16 copy of the hidden layers for SPK_PREC_BF16X3, in the A
  // operand order of the 16x16x32 BF16 MFMA: [t2][tp][lane] = (8 hi, 8 lo)
  // for W[16 tp + c][32 t2 + 8 g + i], i = 0..7 (hi = RNE(W), lo = RNE(W - hi))
  const int MT2 = MT / 2;
  const size_t nWb = (size_t)(L - 2) * H * H * 2;   // uint16 count (hi + lo)
  std::vector<uint16_t> Wb(nWb);
  for (int l = 1; l <= L - 2; ++l) {
    const float* Wl = W[l];
    uint16_t* dst = Wb.data() + (size_t)(l - 1) * H * H * 2;
    for (int t2 = 0; t2 < MT2; ++t2)
      for (int tp = 0; tp < MT; ++tp)
        for (int lane = 0; lane < 64; ++lane) {
          const int g = lane >> 4, c = lane & 15;
          uint16_t* o = dst + (((size_t)t2 * MT + tp) * 64 + lane) * 16;
          for (int i = 0; i < 8; ++i) {
            const float w = Wl[(size_t)(16 * tp + c) * H + 32 * t2 + 8 * g + i];
            const uint16_t hi = bf16_rne(w);
            o[i] = hi;
            o[8 + i] = bf16_rne(w - bf16_to_f32(hi));
          }
        }
  }
  // scaled split-FP16 copy for SPK_PREC_F16X3, same fragment order as the
  // BF16 copy: per layer W' = W 2^sW with max |W'| in [2^14, 2^15),
  // hi = RNE16(W'), lo = RNE16(W' - hi) (no subnormals stored).  The residual
  // dw = W' - hi - lo is exact in FP64 (all three terms are short); it goes
  // to the relative bound cw when |dw| <= 2^-21 |W'|, else to the absolute
  // per-row sum D_j (weights below ~2^-3 in scaled units, whose lo part
  // underflows).
  std::vector<uint16_t> Wh(nWb);
  std::vector<float> wsh((size_t)(L > 2 ? L - 2 : 1), 1.0f), dwt(nbh > 0 ? nbh : 1, 0.0f);
  std::vector<double> Dj((size_t)H);
  double cw = 0.0;
  for (int l = 1; l <= L - 2; ++l) {
    const float* Wl = W[l];
    double m = 0.0;
    for (size_t q = 0; q < (size_t)H * H; ++q) m = fmax(m, fabs((double)Wl[q]));
    int sW = 0;
    if (m > 0.0) {
      int e = 0;
      (void)frexp(m, &e);
      sW = std::min(15 - e, 126);
    }
    wsh[(size_t)(l - 1)] = (float)ldexp(1.0, -sW);
    std::fill(Dj.begin(), Dj.end(), 0.0);
    uint16_t* dst = Wh.data() + (size_t)(l - 1) * H * H * 2;
    for (int t2 = 0; t2 < MT2; ++t2)
      for (int tp = 0; tp < MT; ++tp)
        for (int lane = 0; lane < 64; ++lane) {
          const int g = lane >> 4, c = lane & 15;
          uint16_t* o = dst + (((size_t)t2 * MT + tp) * 64 + lane) * 16;
          for (int i = 0; i < 8; ++i) {
            const double w = ldexp((double)Wl[(size_t)(16 * tp + c) * H + 32 * t2 + 8 * g + i], sW);
            double hv = 0.0, lv = 0.0;
            o[i] = f16_rne_ftz(w, &hv);
            o[8 + i] = f16_rne_ftz(w - hv, &lv);
            const double dw = fabs(w - hv - lv);
            if (dw <= ldexp(fabs(w), -21))
              cw = fmax(cw, dw / fabs(w));
            else
              Dj[(size_t)(16 * tp + c)] += dw;
          }
        }
    // per row: 2^-12 sum_k |W_jk| (X underflow) + D_j 2^(15 - sW) (W residuals)
    for (int r = 0; r < H; ++r) {
      double l1 = 0.0;
      for (int k = 0; k < H; ++k) l1 += fabs((double)Wl[(size_t)r * H + k]);
      dwt[(size_t)(l - 1) * H + r] = up_f32((ldexp(l1, -12) + Dj[(size_t)r] * ldexp(1.0, 15 - sW)) * (1.0 + 1e-6));
    }
  }
  // 4x4 blocks of the hidden layers for row-owner products (packed ray
  // kernel): Wr[l][kb][rb][i][j] = W[4 rb + i][4 kb + j], so lane rb's four
  // rows at one k step are 64 contiguous bytes and a wave's step is one
  // contiguous H*16-byte block
  std::vector<float> Wr(nWp);
  for (int l = 1; l <= L - 2; ++l) {
    float* dst = Wr.data() + (size_t)(l - 1) * H * H;
    for (int kb = 0; kb < H / 4; ++kb)
      for (int rb = 0; rb < H / 4; ++rb)
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j)
            dst[(((size_t)kb * (H / 4) + rb) * 4 + i) * 4 + j] = W[l][(size_t)(4 * rb + i) * H + 4 * kb + j];
  }
  for (int r = 0; r < H; ++r) wL[r] = W[L - 1][r];
  const float bL = b[L - 1][0];

  // one device block, 256-byte aligned pieces
  auto al = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
  const size_t oW0 = 0, ob0 = oW0 + al(nW0 * 4), oWp = ob0 + al(nb0 * 4), obh = oWp + al(nWp * 4 + 4),
               oebh = obh + al(nbh * 4 + 4), owL = oebh + al(nbh * 4 + 4), oWb = owL + al((size_t)H * 4),
               oWr = oWb + al(nWb * 2 + 4), oWh = oWr + al(nWp * 4 + 4), owsh = oWh + al(nWb * 2 + 4),
               odwt = owsh + al(wsh.size() * 4), total = odwt + al(dwt.size() * 4);
  std::vector<unsigned char> img(total, 0);
  memcpy(img.data() + oW0, W0.data(), nW0 * 4);
  memcpy(img.data() + ob0, b0.data(), nb0 * 4);
  if (nWp) memcpy(img.data() + oWp, Wp.data(), nWp * 4);
  if (nbh) {
    memcpy(img.data() + obh, bh.data(), nbh * 4);
    memcpy(img.data() + oebh, ebh.data(), nbh * 4);
  }
  memcpy(img.data() + owL, wL.data(), (size_t)H * 4);
  if (nWb) memcpy(img.data() + oWb, Wb.data(), nWb * 2);
  if (nWp) memcpy(img.data() + oWr, Wr.data(), nWp * 4);
  if (nWb) memcpy(img.data() + oWh, Wh.data(), nWb * 2);
  memcpy(img.data() + owsh, wsh.data(), wsh.size() * 4);
  memcpy(img.data() + odwt, dwt.data(), dwt.size() * 4);

  spk_net* net = new (std::nothrow) spk_net();
  if (net == nullptr) return SPK_E_NOMEM;
  if (hipGetDevice(&net->device) != hipSuccess) { delete net; return SPK_E_DEVICE; }
  void* blk = nullptr;
  if (hipMalloc(&blk, total) != hipSuccess) { delete net; return SPK_E_NOMEM; }
  if (hipMemcpy(blk, img.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(blk);
    delete net;
    return SPK_E_DEVICE;
  }
  unsigned char* base = (unsigned char*)blk;
  NetDev& d = net->dev;
  d.L = L;
  d.H = H;
  d.act = act;
  d.omega0 = act == SPK_ACT_SIN ? omega0 : 1.0f;
  d.cK = up_f32(cK);
  d.cD = up_f32(cD);
  d.c3 = up_f32(c3);
  d.eL = up_f32(cK * fabs((double)bL) + eta);
  d.bL = bL;
  d.W0 = (const float*)(base + oW0);
  d.b0 = (const float*)(base + ob0);
  d.Wp = (const float*)(base + oWp);
  d.bh = (const float*)(base + obh);
  d.ebh = (const float*)(base + oebh);
  d.wL = (const float*)(base + owL);
  d.Wb = (const uint32_t*)(base + oWb);
  d.cKs = up_f32(split_const(H));
  d.Wr = (const float*)(base + oWr);
  d.Wh = (const uint32_t*)(base + oWh);
  d.wsh = (const float*)(base + owsh);
  d.dwt = (const float*)(base + odwt);
  d.cKh = up_f32(split16_const(H, cw));
  net->dev_block = blk;
  net->n_linear = n_linear;
  net->width = H;
  *out = net;
  return SPK_OK;
}

spk_status spk_net_destroy(spk_net* net) {
  if (net == nullptr) return SPK_E_INVAL;
  if (net->holders.load() > 0) return SPK_E_BUSY;
  {
    std::lock_guard<std::mutex> lock(net->use_mu);
    for (auto& u : net->uses)
      if (hipEventQuery(u.second) == hipErrorNotReady) return SPK_E_BUSY;
    for (auto& u : net->uses) (void)hipEventDestroy(u.second);
    net->uses.clear();
  }
  spk_status st = SPK_OK;
  if (net->dev_block) st = check_hip(hipFree(net->dev_block));
  delete net;
  return st;
}

spk_status spk_ctx_create(void* stream, size_t workspace_bytes, spk_ctx** out) {
  if (out == nullptr) return SPK_E_INVAL;
  *out = nullptr;
  spk_ctx* ctx = new (std::nothrow) spk_ctx();
  if (ctx == nullptr) return SPK_E_NOMEM;
  ctx->stream = (hipStream_t)stream;
  ctx->workspace_limit = workspace_bytes;
  ctx->scratch = nullptr;
  ctx->scratch_bytes = 0;
  ctx->status = nullptr;
  ctx->ws_peak = 0;
  if (hipGetDevice(&ctx->device) != hipSuccess ||
      hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) {
    delete ctx;
    return SPK_E_DEVICE;
  }
  if (hipMalloc(&ctx->status, 256) != hipSuccess) {
    delete ctx;
    return SPK_E_NOMEM;
  }
  if (hipMemset(ctx->status, 0, 256) != hipSuccess) {
    (void)hipFree(ctx->status);
    delete ctx;
    return SPK_E_DEVICE;
  }
  *out = ctx;
  return SPK_OK;
}

spk_status spk_ctx_destroy(spk_ctx* ctx) {
  if (ctx == nullptr) return SPK_E_INVAL;
  spk_status st = check_hip(hipStreamSynchronize(ctx->stream));
  if (ctx->scratch && hipFree(ctx->scratch) != hipSuccess) st = SPK_E_DEVICE;
  if (ctx->status && hipFree(ctx->status) != hipSuccess) st = SPK_E_DEVICE;
  delete ctx;
  return st;
}

spk_status spk_ctx_sync(spk_ctx* ctx, spk_device_status* status) {
  if (ctx == nullptr) return SPK_E_INVAL;
  spk_status st = check_hip(hipStreamSynchronize(ctx->stream));
  if (st != SPK_OK) return st;
  spk_device_status ds = {};
  if (hipMemcpy(&ds, ctx->status, sizeof(ds), hipMemcpyDeviceToHost) != hipSuccess) return SPK_E_DEVICE;
  if (hipMemset(ctx->status, 0, sizeof(ds)) != hipSuccess) return SPK_E_DEVICE;
  if (status != nullptr) *status = ds;
  return ds.nospc ? SPK_E_NOSPC : SPK_OK;
}

static spk_status ctx_scratch(spk_ctx* ctx, size_t bytes, void** p) {
  if (bytes > ctx->scratch_bytes) {
    if (ctx->workspace_limit && bytes > ctx->workspace_limit) return SPK_E_NOMEM;
    if (ctx->scratch) {
      if (hipStreamSynchronize(ctx->stream) != hipSuccess) return SPK_E_DEVICE;
      (void)hipFree(ctx->scratch);
      ctx->scratch = nullptr;
      ctx->scratch_bytes = 0;
    }
    const size_t sz = (bytes + 4095) & ~(size_t)4095;
    if (hipMalloc(&ctx->scratch, sz) != hipSuccess) return SPK_E_NOMEM;
    ctx->scratch_bytes = sz;
  }
  *p = ctx->scratch;
  return SPK_OK;
}

static void fill_aux(BoundJob& job, const spk_bound_aux* aux) {
  if (aux) {
    job.center = aux->center;
    job.radius = aux->radius;
    job.err = aux->err;
    job.slot_src = aux->slot_src;
  }
}

spk_status spk_range_bound(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts, int64_t n, int32_t s,
                           const float* center, const float* axes, float* lo, float* hi, const spk_bound_aux* aux) {
  if (ctx == nullptr || net == nullptr) return SPK_E_INVAL;
  spk_status st = valid_opts(opts);
  if (st != SPK_OK) return st;
  if (n < 0 || s < 1 || s > 3) return SPK_E_INVAL;
  if (n == 0) return SPK_OK;
  if (center == nullptr || axes == nullptr || lo == nullptr || hi == nullptr) return SPK_E_INVAL;
  if (aux && aux->slot_src && opts->policy != SPK_AFFINE_TRUNCATE) return SPK_E_INVAL;
  BoundJob job = {};
  job.n = n;
  job.mode = IN_GENERAL;
  job.s = s;
  job.policy = opts->policy;
  job.k = opts->k;
  job.prec = opts->prec;
  job.rigorous = rigorous_opts(opts) ? 1 : 0;
  job.a = center;
  job.b = axes;
  job.lo = lo;
  job.hi = hi;
  job.nonfinite = (unsigned long long*)ctx->status;
  fill_aux(job, aux);
  st = launch_bound(net, job, ctx->stream, ctx->num_cus);
  if (st == SPK_OK) net_mark_use(net, ctx->stream);
  return st;
}

spk_status spk_classify_boxes(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts, int64_t n,
                              const float* box_lo, const float* box_hi, uint8_t* label, float* lo, float* hi,
                              const spk_bound_aux* aux) {
  if (ctx == nullptr || net == nullptr) return SPK_E_INVAL;
  spk_status st = valid_opts(opts);
  if (st != SPK_OK) return st;
  if (n < 0) return SPK_E_INVAL;
  if (n == 0) return SPK_OK;
  if (box_lo == nullptr || box_hi == nullptr || label == nullptr) return SPK_E_INVAL;
  if (aux && aux->slot_src && opts->policy != SPK_AFFINE_TRUNCATE) return SPK_E_INVAL;
  BoundJob job = {};
  job.n = n;
  job.mode = IN_AABB;
  job.s = 3;
  job.policy = opts->policy;
  job.k = opts->k;
  job.prec = opts->prec;
  job.rigorous = rigorous_opts(opts) ? 1 : 0;
  job.a = box_lo;
  job.b = box_hi;
  job.lo = lo;
  job.hi = hi;
  job.label = label;
  job.nonfinite = (unsigned long long*)ctx->status;
  fill_aux(job, aux);
  st = launch_bound(net, job, ctx->stream, ctx->num_cus);
  if (st == SPK_OK) net_mark_use(net, ctx->stream);
  return st;
}

// One frontier round given the per-cell label buffer `labels` (n bytes of
// device memory the call may overwrite).
// Whether the convergence test applies at `level`: the cells' widest side is
// below delta / sqrt(3).
static bool converge_level(const spk_tree_params* tree, int32_t level) {
  if (!(tree->delta > 0.0f)) return false;
  double side = 0.0;
  for (int d = 0; d < 3; ++d)
    side = fmax(side, ((double)tree->dom_hi[d] - (double)tree->dom_lo[d]) / (double)(1u << level));
  return side < (double)tree->delta / 1.7320508075688772;
}

// `faces` (nullable): 96 bytes per cell for the convergence test.
static spk_status subdivide_round(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                                  const spk_tree_params* tree, int32_t level, const uint64_t* cells, int64_t n,
                                  uint64_t* children, int64_t cap_children, uint64_t* leaves, int64_t cap_leaves,
                                  int64_t* counts, uint8_t* labels, float* faces = nullptr) {
  BoundJob job = {};
  job.n = n;
  job.mode = IN_CELL;
  job.s = 3;
  job.policy = opts->policy;
  job.k = opts->k;
  job.prec = opts->prec;
  job.rigorous = rigorous_opts(opts) ? 1 : 0;
  job.cells = cells;
  job.level = level;
  for (int d = 0; d < 3; ++d) {
    job.dom_lo[d] = tree->dom_lo[d];
    job.dom_hi[d] = tree->dom_hi[d];
  }
  job.label = labels;
  job.nonfinite = (unsigned long long*)ctx->status;
  job.band = tree->band;
  if (n > 0) {
    spk_status st = launch_bound(net, job, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    if (faces != nullptr) {
      st = launch_converge(net, labels, cells, n, level, tree->dom_lo, tree->dom_hi, faces, faces + 18 * n,
                           ctx->stream, ctx->num_cus);
      if (st != SPK_OK) return st;
    }
  }
  return launch_compact(labels, cells, n, level == tree->max_level, children, cap_children, leaves, cap_leaves,
                        counts, ctx->status, ctx->stream, ctx->num_cus);
}

static spk_status check_subdivide_args(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                                       const spk_tree_params* tree, int32_t level, const uint64_t* cells, int64_t n,
                                       const uint64_t* children, int64_t cap_children, const uint64_t* leaves,
                                       int64_t cap_leaves, const int64_t* counts) {
  if (ctx == nullptr || net == nullptr || tree == nullptr || counts == nullptr) return SPK_E_INVAL;
  spk_status st = valid_opts(opts);
  if (st != SPK_OK) return st;
  if (tree->arity != 8) return SPK_E_UNSUPPORTED;
  if (tree->max_level < 0 || tree->max_level > 20 || level < 0 || level > tree->max_level) return SPK_E_INVAL;
  for (int d = 0; d < 3; ++d)
    if (!(tree->dom_lo[d] < tree->dom_hi[d]) || !isfinite(tree->dom_lo[d]) || !isfinite(tree->dom_hi[d]))
      return SPK_E_INVAL;
  if (!(tree->delta >= 0.0f) || !isfinite(tree->delta)) return SPK_E_INVAL;
  if (!(tree->band >= 0.0f) || !isfinite(tree->band) || (tree->band > 0.0f && tree->delta > 0.0f)) return SPK_E_INVAL;
  if (n < 0 || cap_children < 0 || cap_leaves < 0) return SPK_E_INVAL;
  if (n > 0 && cells == nullptr) return SPK_E_INVAL;
  if ((cap_children > 0 && children == nullptr) || (cap_leaves > 0 && leaves == nullptr)) return SPK_E_INVAL;
  return SPK_OK;
}

spk_status spk_subdivide_frontier(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                                  const spk_tree_params* tree, int32_t level, const uint64_t* cells, int64_t n,
                                  uint64_t* children, int64_t cap_children, uint64_t* leaves, int64_t cap_leaves,
                                  int64_t* counts) {
  spk_status st = check_subdivide_args(ctx, net, opts, tree, level, cells, n, children, cap_children, leaves,
                                       cap_leaves, counts);
  if (st != SPK_OK) return st;
  void* labels = nullptr;
  float* faces = nullptr;
  if (n > 0) {
    // labels, then (for the convergence test) 18 face coordinates and 6
    // values per cell
    const bool conv = converge_level(tree, level);
    const size_t lab_bytes = ((size_t)n + 255) & ~(size_t)255;
    st = ctx_scratch(ctx, lab_bytes + (conv ? (size_t)n * 96 : 0), &labels);
    if (st != SPK_OK) return st;
    if (conv) faces = (float*)((char*)labels + lab_bytes);
  }
  st = subdivide_round(ctx, net, opts, tree, level, cells, n, children, cap_children, leaves, cap_leaves, counts,
                       (uint8_t*)labels, faces);
  if (st == SPK_OK) net_mark_use(net, ctx->stream);
  return st;
}

spk_status spk_subdivide_frontier_noalloc(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                                          const spk_tree_params* tree, int32_t level, const uint64_t* cells,
                                          int64_t n, uint64_t* children, int64_t cap_children, uint64_t* leaves,
                                          int64_t cap_leaves, int64_t* counts) {
  spk_status st = check_subdivide_args(ctx, net, opts, tree, level, cells, n, children, cap_children, leaves,
                                       cap_leaves, counts);
  if (st != SPK_OK) return st;
  if (tree->delta != 0.0f) return SPK_E_UNSUPPORTED;   // its face buffers would need an allocation
  if (opts->policy == SPK_AFFINE_FULL) return SPK_E_UNSUPPORTED;   // so would affine-full's workspace
  if (n > (int64_t)SPK_NOALLOC_MAX_CELLS) return SPK_E_LIMIT;
  void* labels = nullptr;
  st = noalloc_scratch(ctx->device, &labels);
  if (st != SPK_OK) return st;
  return subdivide_round(ctx, net, opts, tree, level, cells, n, children, cap_children, leaves, cap_leaves, counts,
                         (uint8_t*)labels);
}

spk_status spk_cast_rays(spk_ctx* ctx, const spk_net* net, const spk_ray_params* params, int64_t n,
                         const float* origin, const float* dir, float* t_hit, int32_t* iters) {
  if (ctx == nullptr || net == nullptr || params == nullptr) return SPK_E_INVAL;
  if (n < 0) return SPK_E_INVAL;
  const spk_ray_params& p = *params;
  if (!(p.delta > 0.0f) || !(p.sigma0 > 0.0f) || !(p.eta_minus > 0.0f && p.eta_minus < 1.0f) ||
      !(p.eta_plus >= 1.0f) || !(p.safety > 0.0f && p.safety <= 1.0f) || p.max_iters <= 0 ||
      !isfinite(p.delta) || !isfinite(p.sigma0) || !isfinite(p.eta_plus))
    return SPK_E_INVAL;
  if (!p.clip_to_domain && !(p.t_max > 0.0f && isfinite(p.t_max))) return SPK_E_INVAL;
  if (p.flags & ~(uint32_t)SPK_FLAG_NO_ROUNDING_BOUND) return SPK_E_INVAL;
  if (n == 0) return SPK_OK;
  if (origin == nullptr || dir == nullptr || t_hit == nullptr) return SPK_E_INVAL;
  void* counter = nullptr;
  spk_status st = ctx_scratch(ctx, 256, &counter);
  if (st != SPK_OK) return st;
  st = launch_rays(net, p, n, origin, dir, t_hit, iters, (unsigned long long*)counter, ctx->stream, ctx->num_cus);
  if (st == SPK_OK) net_mark_use(net, ctx->stream);
  return st;
}

namespace {
// Device buffers owned by one closest-point call, allocated stream-ordered
// on the context's stream (hipMallocAsync / hipFreeAsync), so that growing or
// releasing them neither waits for the device nor stalls other streams.
struct CallBuffers {
  std::vector<std::pair<void**, size_t>> held;
  size_t total = 0;
  size_t limit = 0;
  size_t* peak = nullptr;   // largest total of the call (nullable)
  hipStream_t stream = nullptr;
  ~CallBuffers() {
    // ordered after every kernel of the call on the stream
    for (auto& h : held)
      if (*h.first) (void)hipFreeAsync(*h.first, stream);
  }
  // Free *p (stream-ordered after the call's earlier launches).
  void release(void** p, size_t& cap) {
    if (*p) (void)hipFreeAsync(*p, stream);
    *p = nullptr;
    total -= cap;
    cap = 0;
  }
  // (Re)allocate *p to at least `bytes`; contents are not kept.
  spk_status ensure(void** p, size_t& cap, size_t bytes) {
    if (bytes <= cap) return SPK_OK;
    const size_t want = bytes + bytes / 2;
    if (limit && total - cap + want > limit) return SPK_E_NOMEM;
    // earlier launches of the call on the stream still read the old buffer:
    // the stream-ordered free runs after them
    if (*p) (void)hipFreeAsync(*p, stream);
    *p = nullptr;
    total -= cap;
    cap = 0;
    if (hipMallocAsync(p, want, stream) != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();   // clear it, so that later launch checks do not report it
      return SPK_E_NOMEM;
    }
    cap = want;
    total += want;
    if (peak && total > *peak) *peak = total;
    bool known = false;
    for (auto& h : held) known = known || h.first == p;
    if (!known) held.push_back({p, 0});
    return SPK_OK;
  }
};
}  // namespace

// One chunk of queries through every level (see spk_closest_point); the
// buffers are reused from chunk to chunk.
struct CpBuffers {
  void *best = nullptr, *codes = nullptr, *qidx = nullptr, *ncodes = nullptr, *nqidx = nullptr, *labels = nullptr,
       *fpts = nullptr, *fvals = nullptr, *cnt = nullptr, *dcur = nullptr;
  size_t c_best = 0, c_codes = 0, c_qidx = 0, c_ncodes = 0, c_nqidx = 0, c_labels = 0, c_fpts = 0, c_fvals = 0,
         c_cnt = 0, c_dcur = 0;
  // distinct cells of a round: sorted codes, distinct codes, their labels and
  // face values, the sort / unique temporary storage
  void *sorted = nullptr, *ucodes = nullptr, *ulabels = nullptr, *ufvals = nullptr, *dtemp = nullptr;
  size_t c_sorted = 0, c_ucodes = 0, c_ulabels = 0, c_ufvals = 0, c_dtemp = 0;
  CallBuffers B;   // last: destroyed first, while the pointers above are alive
};

// Rounds with at least this many (query, cell) items classify each distinct
// cell once (sort + unique + gather); below it the items are bounded directly.
constexpr int64_t kCpShareMin = 4096;

static spk_status closest_chunk(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                                const spk_tree_params* tree, int64_t n, const float* q, float* point, float* dist,
                                float* bound, CpBuffers& CB) {
  CallBuffers& B = CB.B;
  void*& best = CB.best;
  void*& codes = CB.codes;
  void*& qidx = CB.qidx;
  void*& ncodes = CB.ncodes;
  void*& nqidx = CB.nqidx;
  void*& labels = CB.labels;
  void*& fpts = CB.fpts;
  void*& fvals = CB.fvals;
  void*& cnt = CB.cnt;
  void*& dcur = CB.dcur;
  size_t& c_best = CB.c_best;
  size_t& c_codes = CB.c_codes;
  size_t& c_qidx = CB.c_qidx;
  size_t& c_ncodes = CB.c_ncodes;
  size_t& c_nqidx = CB.c_nqidx;
  size_t& c_labels = CB.c_labels;
  size_t& c_fpts = CB.c_fpts;
  size_t& c_fvals = CB.c_fvals;
  size_t& c_cnt = CB.c_cnt;
  spk_status st = SPK_OK;
#define SPK_ENSURE(ptr, cap, bytes)                 \
  do {                                              \
    spk_status e_ = B.ensure(&(ptr), cap, (bytes)); \
    if (e_ != SPK_OK) return e_;                    \
  } while (0)
  SPK_ENSURE(best, c_best, (size_t)n * 4);
  SPK_ENSURE(codes, c_codes, (size_t)n * 8);
  SPK_ENSURE(qidx, c_qidx, (size_t)n * 4);
  SPK_ENSURE(cnt, c_cnt, 256);
  st = launch_cp_init(n, (uint64_t*)codes, (uint32_t*)qidx, (unsigned*)best, point, ctx->stream, ctx->num_cus);
  if (st != SPK_OK) return st;
  if (rigorous_opts(opts) && tree->max_level >= 1) {
    // seeding descent (closest.hip): under sound bounds every cell it uses is
    // one the level rounds would reach, so the result does not change; the
    // frontier buffers of the rounds serve as its child buffers
    SPK_ENSURE(dcur, CB.c_dcur, (size_t)n * 8);
    SPK_ENSURE(ncodes, c_ncodes, (size_t)n * 8 * 8);
    SPK_ENSURE(labels, c_labels, (size_t)n * 8);
    SPK_ENSURE(fpts, c_fpts, (size_t)n * 48 * 12);
    SPK_ENSURE(fvals, c_fvals, (size_t)n * 48 * 4);
    st = launch_cp_dive_init(n, (uint64_t*)dcur, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    for (int level = 1; level <= tree->max_level; ++level) {
      CpDive D = {};
      D.n = n;
      D.level = level;
      for (int d = 0; d < 3; ++d) {
        D.dom_lo[d] = tree->dom_lo[d];
        D.dom_hi[d] = tree->dom_hi[d];
      }
      D.q = q;
      D.cur = (uint64_t*)dcur;
      D.codes = (uint64_t*)ncodes;
      D.label = (const uint8_t*)labels;
      D.fpts = (float*)fpts;
      D.fvals = (const float*)fvals;
      D.best = (unsigned*)best;
      D.point = point;
      st = launch_cp_dive_children(D, ctx->stream, ctx->num_cus);
      if (st != SPK_OK) return st;
      BoundJob job = {};
      job.n = 8 * n;
      job.mode = IN_CELL;
      job.s = 3;
      job.policy = opts->policy;
      job.k = opts->k;
      job.prec = opts->prec;
      job.rigorous = 1;
      job.cells = (const uint64_t*)ncodes;
      job.level = level;
      for (int d = 0; d < 3; ++d) {
        job.dom_lo[d] = tree->dom_lo[d];
        job.dom_hi[d] = tree->dom_hi[d];
      }
      job.label = (uint8_t*)labels;
      st = launch_bound(net, job, ctx->stream, ctx->num_cus);
      if (st != SPK_OK) return st;
      st = launch_eval(net, 48 * n, (const float*)fpts, (float*)fvals, ctx->stream, ctx->num_cus);
      if (st != SPK_OK) return st;
      st = launch_cp_dive_pick(D, ctx->stream, ctx->num_cus);
      if (st != SPK_OK) return st;
    }
  }
  int64_t m = n;
  for (int level = 0; level <= tree->max_level && m > 0; ++level) {
    const bool at_max = level == tree->max_level;
    SPK_ENSURE(labels, c_labels, (size_t)m);
    SPK_ENSURE(fpts, c_fpts, (size_t)m * 18 * 4);
    SPK_ENSURE(fvals, c_fvals, (size_t)m * 6 * 4);
    if (!at_max) {
      SPK_ENSURE(ncodes, c_ncodes, (size_t)m * 8 * 8);
      SPK_ENSURE(nqidx, c_nqidx, (size_t)m * 8 * 4);
    }
    BoundJob job = {};
    job.n = m;
    job.mode = IN_CELL;
    job.s = 3;
    job.policy = opts->policy;
    job.k = opts->k;
    job.prec = opts->prec;
    job.rigorous = rigorous_opts(opts) ? 1 : 0;
    job.cells = (const uint64_t*)codes;
    job.level = level;
    for (int d = 0; d < 3; ++d) {
      job.dom_lo[d] = tree->dom_lo[d];
      job.dom_hi[d] = tree->dom_hi[d];
    }
    job.label = (uint8_t*)labels;
    job.nonfinite = (unsigned long long*)ctx->status;
    // large rounds: classify and evaluate each distinct cell once, when the
    // workspace limit leaves room for the sort (else every item is bounded)
    bool shared = m >= kCpShareMin && m <= (int64_t)0x7fffffff;   // the sort counts items in 32 bits
    int64_t nu = 0;
    if (shared) {
      const size_t tb = cp_dedup_temp_bytes(m);
      shared = B.ensure(&CB.sorted, CB.c_sorted, (size_t)m * 8) == SPK_OK &&
               B.ensure(&CB.ucodes, CB.c_ucodes, (size_t)m * 8) == SPK_OK &&
               B.ensure(&CB.dtemp, CB.c_dtemp, tb) == SPK_OK &&
               B.ensure(&CB.ulabels, CB.c_ulabels, (size_t)m) == SPK_OK &&
               B.ensure(&CB.ufvals, CB.c_ufvals, (size_t)m * 6 * 4) == SPK_OK;
      if (!shared) {
        // give the room back to the frontier buffers
        B.release(&CB.sorted, CB.c_sorted);
        B.release(&CB.ucodes, CB.c_ucodes);
        B.release(&CB.dtemp, CB.c_dtemp);
        B.release(&CB.ulabels, CB.c_ulabels);
        B.release(&CB.ufvals, CB.c_ufvals);
      }
    }
    if (shared) {
      int64_t* dnu = (int64_t*)((char*)cnt + 64);
      st = launch_cp_dedup((const uint64_t*)codes, (uint64_t*)CB.sorted, (uint64_t*)CB.ucodes, dnu, m, level,
                           CB.dtemp, CB.c_dtemp, ctx->stream);
      if (st != SPK_OK) return st;
      if (hipMemcpyAsync(&nu, dnu, sizeof(nu), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess)
        return SPK_E_DEVICE;
      if (nu < 1 || nu > m) return SPK_E_DEVICE;
      job.n = nu;
      job.cells = (const uint64_t*)CB.ucodes;
      job.label = (uint8_t*)CB.ulabels;
    }
    st = launch_bound(net, job, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    CpLevel L = {};
    L.m = m;
    L.level = level;
    L.at_max = at_max ? 1 : 0;
    L.shared = shared ? 1 : 0;
    for (int d = 0; d < 3; ++d) {
      L.dom_lo[d] = tree->dom_lo[d];
      L.dom_hi[d] = tree->dom_hi[d];
    }
    L.codes = (const uint64_t*)codes;
    L.qidx = (const uint32_t*)qidx;
    L.label = (const uint8_t*)labels;
    L.q = q;
    L.best = (unsigned*)best;
    L.point = point;
    L.fpts = (float*)fpts;
    L.fvals = (float*)fvals;
    L.ncodes = (uint64_t*)ncodes;
    L.nqidx = (uint32_t*)nqidx;
    L.ncount = (unsigned long long*)cnt;
    L.cap = at_max ? 0 : m * 8;
    if (shared) {
      // face centers of the distinct cells in fpts (nu <= m), their values in
      // ufvals, gathered into every item's labels and fvals
      CpLevel U = L;
      U.m = nu;
      U.codes = (const uint64_t*)CB.ucodes;
      st = launch_cp_shared(net, U, (const uint64_t*)codes, m, (const uint8_t*)CB.ulabels, (float*)CB.ufvals,
                            (uint8_t*)labels, (float*)fvals, ctx->stream, ctx->num_cus);
      if (st != SPK_OK) return st;
    }
    st = launch_cp_round(net, L, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    if (at_max) break;
    unsigned long long next = 0ull;
    if (hipMemcpyAsync(&next, cnt, sizeof(next), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return SPK_E_DEVICE;
    m = (int64_t)next;   // at most 8 m by construction
    std::swap(codes, ncodes);
    std::swap(c_codes, c_ncodes);
    std::swap(qidx, nqidx);
    std::swap(c_qidx, c_nqidx);
  }
#undef SPK_ENSURE
  return launch_cp_finish(n, q, (const unsigned*)best, point, dist, bound, ctx->stream, ctx->num_cus);
}


spk_status spk_closest_point(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                             const spk_tree_params* tree, int64_t n, const float* q, float* point, float* dist,
                             float* bound) {
  if (ctx == nullptr || net == nullptr || tree == nullptr) return SPK_E_INVAL;
  spk_status st = valid_opts(opts);
  if (st != SPK_OK) return st;
  if (tree->arity != 8) return SPK_E_UNSUPPORTED;
  if (tree->max_level < 0 || tree->max_level > 20 || tree->delta != 0.0f || tree->band != 0.0f) return SPK_E_INVAL;
  for (int d = 0; d < 3; ++d)
    if (!(tree->dom_lo[d] < tree->dom_hi[d]) || !isfinite(tree->dom_lo[d]) || !isfinite(tree->dom_hi[d]))
      return SPK_E_INVAL;
  if (n < 0 || n > (int64_t)0xffffffffLL) return SPK_E_INVAL;
  if (n == 0) return SPK_OK;
  if (q == nullptr || point == nullptr) return SPK_E_INVAL;

  // queries run in chunks so that the frontier memory stays bounded; a chunk
  // whose frontier outgrows the workspace limit is retried in halves (each
  // chunk starts from the root, so a retry recomputes it in full)
  int64_t chunk = 1024;
  CpBuffers CB;
  CB.B.limit = ctx->workspace_limit ? ctx->workspace_limit : ((size_t)16 << 30);
  CB.B.stream = ctx->stream;
  CB.B.peak = &ctx->ws_peak;
  for (int64_t c0 = 0; c0 < n;) {
    const int64_t cn = (n - c0 < chunk) ? n - c0 : chunk;
    st = closest_chunk(ctx, net, opts, tree, cn, q + 3 * c0, point + 3 * c0, dist ? dist + c0 : nullptr,
                       bound ? bound + c0 : nullptr, CB);
    if (st == SPK_E_NOMEM && cn > 1) {
      chunk = (cn + 1) / 2;
      continue;
    }
    if (st != SPK_OK) return st;
    c0 += cn;
  }
  return check_hip(hipStreamSynchronize(ctx->stream));
}

// Sampling in leaf cells (Sections 4.6, 4.8); kernels in samples.hip.
spk_status spk_sample_leaves(spk_ctx* ctx, const spk_net* net, const spk_tree_params* tree, int32_t level,
                             int64_t n_leaves, const uint64_t* leaves, int64_t n_samples, uint64_t seed, float band,
                             float* points, float* f, int64_t cap, int64_t* n_accepted, int64_t* n_below) {
  if (ctx == nullptr || net == nullptr || tree == nullptr || n_accepted == nullptr) return SPK_E_INVAL;
  if (tree->arity != 8) return SPK_E_UNSUPPORTED;
  for (int d = 0; d < 3; ++d)
    if (!(tree->dom_lo[d] < tree->dom_hi[d]) || !isfinite(tree->dom_lo[d]) || !isfinite(tree->dom_hi[d]))
      return SPK_E_INVAL;
  if (level < 0 || level > 20 || n_leaves < 0 || n_samples < 0 || cap < 0 || !(band > 0.0f)) return SPK_E_INVAL;
  if ((n_leaves > 0 && leaves == nullptr) || (cap > 0 && points == nullptr)) return SPK_E_INVAL;
  if (n_samples > 0 && n_leaves == 0) return SPK_E_INVAL;
  *n_accepted = 0;
  if (n_below) *n_below = 0;
  if (n_samples == 0) return SPK_OK;
  void *pts = nullptr, *vals = nullptr, *cnt = nullptr;
  size_t c_pts = 0, c_vals = 0, c_cnt = 0;
  CallBuffers B;
  B.limit = ctx->workspace_limit;
  B.stream = ctx->stream;
  B.peak = &ctx->ws_peak;
  const int64_t chunk = std::min<int64_t>(n_samples, (int64_t)1 << 24);
  spk_status st = B.ensure(&pts, c_pts, (size_t)chunk * 12);
  if (st == SPK_OK) st = B.ensure(&vals, c_vals, (size_t)chunk * 4);
  if (st == SPK_OK) st = B.ensure(&cnt, c_cnt, 256);
  if (st != SPK_OK) return st;
  if (hipMemsetAsync(cnt, 0, 16, ctx->stream) != hipSuccess) return SPK_E_DEVICE;
  SampleJob J = {};
  J.leaves = leaves;
  J.n_leaves = n_leaves;
  J.level = level;
  for (int d = 0; d < 3; ++d) {
    J.dom_lo[d] = tree->dom_lo[d];
    J.dom_hi[d] = tree->dom_hi[d];
  }
  J.seed = seed;
  J.band = band;
  J.points = points;
  J.f = f;
  J.cap = cap;
  J.counts = (unsigned long long*)cnt;
  for (int64_t i0 = 0; i0 < n_samples; i0 += chunk) {
    st = launch_sample_chunk(net, J, i0, std::min(chunk, n_samples - i0), (float*)pts, (float*)vals, ctx->stream,
                             ctx->num_cus);
    if (st != SPK_OK) return st;
  }
  unsigned long long c[2] = {0ull, 0ull};
  if (hipMemcpyAsync(c, cnt, sizeof(c), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return SPK_E_DEVICE;
  *n_accepted = (int64_t)c[0];
  if (n_below) *n_below = (int64_t)c[1];
  net_mark_use(net, ctx->stream);
  // points == NULL: the counts alone were asked for
  return (points != nullptr && (int64_t)c[0] > cap) ? SPK_E_NOSPC : SPK_OK;
}

// Mesh extraction in leaf cells (Section 4.7); kernels in mesh.hip.
spk_status spk_mesh_leaves(spk_ctx* ctx, const spk_net* net, const spk_tree_params* tree, int32_t level,
                           int32_t dense_levels, int64_t n_leaves, const uint64_t* leaves, float* tris,
                           int32_t* tri_src, int64_t cap_tris, int64_t* n_tris) {
  if (ctx == nullptr || net == nullptr || tree == nullptr || n_tris == nullptr) return SPK_E_INVAL;
  if (tree->arity != 8) return SPK_E_UNSUPPORTED;
  for (int d = 0; d < 3; ++d)
    if (!(tree->dom_lo[d] < tree->dom_hi[d]) || !isfinite(tree->dom_lo[d]) || !isfinite(tree->dom_hi[d]))
      return SPK_E_INVAL;
  if (level < 0 || dense_levels < 0 || dense_levels > 4 || level + dense_levels > 20) return SPK_E_INVAL;
  if (n_leaves < 0 || n_leaves > (int64_t)0x7fffffff || cap_tris < 0) return SPK_E_INVAL;
  if ((n_leaves > 0 && leaves == nullptr) || (cap_tris > 0 && tris == nullptr)) return SPK_E_INVAL;
  *n_tris = 0;
  if (n_leaves == 0) return SPK_OK;
  const int R = 1 << dense_levels, NV = (R + 1) * (R + 1) * (R + 1);
  void *pts = nullptr, *vals = nullptr, *cnt = nullptr;
  size_t c_pts = 0, c_vals = 0, c_cnt = 0;
  CallBuffers B;
  B.limit = ctx->workspace_limit;
  B.stream = ctx->stream;
  B.peak = &ctx->ws_peak;
  // chunks of leaves whose grid points take at most 256 MiB
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_leaves, ((int64_t)256 << 20) / ((int64_t)NV * 16)));
  spk_status st = B.ensure(&pts, c_pts, (size_t)chunk * NV * 12);
  if (st == SPK_OK) st = B.ensure(&vals, c_vals, (size_t)chunk * NV * 4);
  if (st == SPK_OK) st = B.ensure(&cnt, c_cnt, 256);
  if (st != SPK_OK) return st;
  if (hipMemsetAsync(cnt, 0, 8, ctx->stream) != hipSuccess) return SPK_E_DEVICE;
  MeshJob M = {};
  M.leaves = leaves;
  M.level = level;
  M.dense = dense_levels;
  for (int d = 0; d < 3; ++d) {
    M.dom_lo[d] = tree->dom_lo[d];
    M.h[d] = (float)(((double)tree->dom_hi[d] - (double)tree->dom_lo[d]) / (double)(1u << (level + dense_levels)));
  }
  M.tris = tris;
  M.src = tri_src;
  M.cap = cap_tris;
  M.count = (unsigned long long*)cnt;
  for (int64_t l0 = 0; l0 < n_leaves; l0 += chunk) {
    const int64_t nl = std::min(chunk, n_leaves - l0);
    st = launch_mesh_chunk(net, M, l0, nl, (float*)pts, (float*)vals, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
  }
  unsigned long long total = 0ull;
  if (hipMemcpyAsync(&total, cnt, sizeof(total), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return SPK_E_DEVICE;
  *n_tris = (int64_t)total;
  net_mark_use(net, ctx->stream);
  return (int64_t)total > cap_tris ? SPK_E_NOSPC : SPK_OK;
}

// Intersection of two shapes (Section 4.9); the combine kernel is in
// intersect.hip.
spk_status spk_intersect(spk_ctx* ctx, const spk_net* net_f, const spk_net* net_g, const spk_bound_opts* opts,
                         const spk_tree_params* tree, spk_intersect_result* out) {
  if (ctx == nullptr || net_f == nullptr || net_g == nullptr || tree == nullptr || out == nullptr) return SPK_E_INVAL;
  spk_status st = valid_opts(opts);
  if (st != SPK_OK) return st;
  if (tree->arity != 8) return SPK_E_UNSUPPORTED;
  if (tree->max_level < 0 || tree->max_level > 20 || tree->delta != 0.0f || tree->band != 0.0f) return SPK_E_INVAL;
  for (int d = 0; d < 3; ++d)
    if (!(tree->dom_lo[d] < tree->dom_hi[d]) || !isfinite(tree->dom_lo[d]) || !isfinite(tree->dom_hi[d]))
      return SPK_E_INVAL;
  void *cells = nullptr, *kids = nullptr, *lf = nullptr, *lg = nullptr, *cnt = nullptr;
  size_t c_cells = 0, c_kids = 0, c_lf = 0, c_lg = 0, c_cnt = 0;
  CallBuffers B;
  B.limit = ctx->workspace_limit;
  B.stream = ctx->stream;
  B.peak = &ctx->ws_peak;
#define SPK_IX_ENSURE(ptr, cap, bytes)              \
  do {                                              \
    spk_status e_ = B.ensure(&(ptr), cap, (bytes)); \
    if (e_ != SPK_OK) return e_;                    \
  } while (0)
  SPK_IX_ENSURE(cells, c_cells, 8);
  SPK_IX_ENSURE(cnt, c_cnt, 256);
  if (hipMemsetAsync(cells, 0, 8, ctx->stream) != hipSuccess) return SPK_E_DEVICE;   // the root
  *out = spk_intersect_result{};
  out->result = SPK_NO_INTERSECTION;
  out->level = -1;
  int64_t m = 1;
  for (int level = 0; level <= tree->max_level; ++level) {
    const bool at_max = level == tree->max_level;
    SPK_IX_ENSURE(lf, c_lf, (size_t)m);
    SPK_IX_ENSURE(lg, c_lg, (size_t)m);
    if (!at_max) SPK_IX_ENSURE(kids, c_kids, (size_t)m * 64);
    for (int w = 0; w < 2; ++w) {
      BoundJob job = {};
      job.n = m;
      job.mode = IN_CELL;
      job.s = 3;
      job.policy = opts->policy;
      job.k = opts->k;
      job.prec = opts->prec;
      job.rigorous = rigorous_opts(opts) ? 1 : 0;
      job.cells = (const uint64_t*)cells;
      job.level = level;
      for (int d = 0; d < 3; ++d) {
        job.dom_lo[d] = tree->dom_lo[d];
        job.dom_hi[d] = tree->dom_hi[d];
      }
      job.label = (uint8_t*)(w == 0 ? lf : lg);
      st = launch_bound(w == 0 ? net_f : net_g, job, ctx->stream, ctx->num_cus);
      if (st != SPK_OK) return st;
    }
    IxRound X = {};
    X.n = m;
    X.at_max = at_max ? 1 : 0;
    X.cells = (const uint64_t*)cells;
    X.lab_f = (const uint8_t*)lf;
    X.lab_g = (const uint8_t*)lg;
    X.children = (uint64_t*)kids;
    X.cap = at_max ? 0 : m * 8;
    X.counts = (unsigned long long*)cnt;
    st = launch_ix_round(X, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    unsigned long long c[4] = {0ull, 0ull, 0ull, 0ull};
    if (hipMemcpyAsync(c, cnt, sizeof(c), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return SPK_E_DEVICE;
    out->cells_bounded += 2 * m;
    out->rounds = level + 1;
    if (c[3] > 0) {
      out->result = SPK_INTERSECTION;
      out->level = level;
      out->cell = c[2];
      break;
    }
    if (at_max) {
      out->undecided = (int64_t)c[1];
      out->result = c[1] > 0 ? SPK_INTERSECTION_UNDECIDED : SPK_NO_INTERSECTION;
      break;
    }
    if (c[0] == 0) break;   // every cell dropped
    m = (int64_t)c[0];
    std::swap(cells, kids);
    std::swap(c_cells, c_kids);
  }
#undef SPK_IX_ENSURE
  net_mark_use(net_f, ctx->stream);
  net_mark_use(net_g, ctx->stream);
  return SPK_OK;
}

// Empty spheres (Section 4.4); kernels in spheres.hip.
spk_status spk_empty_spheres(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts, int64_t n, const float* p,
                             float r0, float r_min, float* radius, uint8_t* label) {
  if (ctx == nullptr || net == nullptr) return SPK_E_INVAL;
  spk_status st = valid_opts(opts);
  if (st != SPK_OK) return st;
  if (n < 0 || !(r0 > 0.0f) || !(r_min > 0.0f) || !(r_min <= r0) || !isfinite(r0)) return SPK_E_INVAL;
  if (n == 0) return SPK_OK;
  if (p == nullptr || radius == nullptr || label == nullptr) return SPK_E_INVAL;
  void *cur = nullptr, *rc = nullptr, *lc = nullptr, *nx = nullptr, *rn = nullptr, *cnt = nullptr, *blo = nullptr,
       *bhi = nullptr;
  size_t c_cur = 0, c_rc = 0, c_lc = 0, c_nx = 0, c_rn = 0, c_cnt = 0, c_blo = 0, c_bhi = 0;
  CallBuffers B;
  B.limit = ctx->workspace_limit;
  B.stream = ctx->stream;
  B.peak = &ctx->ws_peak;
#define SPK_ES_ENSURE(ptr, cap, bytes)              \
  do {                                              \
    spk_status e_ = B.ensure(&(ptr), cap, (bytes)); \
    if (e_ != SPK_OK) return e_;                    \
  } while (0)
  SPK_ES_ENSURE(cur, c_cur, (size_t)n * 8);
  SPK_ES_ENSURE(rc, c_rc, (size_t)n * 4);
  SPK_ES_ENSURE(lc, c_lc, (size_t)n);
  SPK_ES_ENSURE(nx, c_nx, (size_t)n * 8);
  SPK_ES_ENSURE(rn, c_rn, (size_t)n * 4);
  SPK_ES_ENSURE(cnt, c_cnt, 256);
  SPK_ES_ENSURE(blo, c_blo, (size_t)n * 12);
  SPK_ES_ENSURE(bhi, c_bhi, (size_t)n * 12);
#undef SPK_ES_ENSURE
  EsRound E = {};
  E.n = n;
  E.p = p;
  E.r0 = r0;
  E.r_min = r_min;
  E.cur = (int64_t*)cur;
  E.r_cur = (float*)rc;
  E.lab_cur = (const uint8_t*)lc;
  E.next = (int64_t*)nx;
  E.r_next = (float*)rn;
  E.count = (unsigned long long*)cnt;
  E.box_lo = (float*)blo;
  E.box_hi = (float*)bhi;
  E.radius = radius;
  E.label = label;
  st = launch_es_init(E, ctx->stream);
  if (st != SPK_OK) return st;
  int64_t m = n;
  for (int round = 0; m > 0; ++round) {
    if (round > 200) return SPK_E_DEVICE;   // not reached: r halves each round down to r_min
    st = launch_es_boxes(E, m, ctx->stream);
    if (st != SPK_OK) return st;
    BoundJob job = {};
    job.n = m;
    job.mode = IN_AABB;
    job.s = 3;
    job.policy = opts->policy;
    job.k = opts->k;
    job.prec = opts->prec;
    job.rigorous = rigorous_opts(opts) ? 1 : 0;
    job.a = E.box_lo;
    job.b = E.box_hi;
    job.label = (uint8_t*)lc;
    job.nonfinite = (unsigned long long*)ctx->status;
    st = launch_bound(net, job, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    st = launch_es_update(E, m, ctx->stream);
    if (st != SPK_OK) return st;
    unsigned long long next = 0ull;
    if (hipMemcpyAsync(&next, cnt, sizeof(next), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return SPK_E_DEVICE;
    m = (int64_t)next;
    if (m > n) return SPK_E_DEVICE;
    std::swap(E.cur, E.next);
    std::swap(E.r_cur, E.r_next);
  }
  return check_hip(hipStreamSynchronize(ctx->stream));
}

// Frustum ray casting (Section 4.3; Appendix B); kernels in frustum.hip.
spk_status spk_cast_frusta(spk_ctx* ctx, const spk_net* net, const spk_ray_params* params,
                           const spk_bound_opts* box_opts, const spk_camera* cam, int32_t tiles_x, int32_t tiles_y,
                           float* t_hit, int32_t* iters, spk_frustum_stats* stats) {
  if (ctx == nullptr || net == nullptr || params == nullptr || cam == nullptr) return SPK_E_INVAL;
  spk_status st = valid_opts(box_opts);
  if (st != SPK_OK) return st;
  const spk_ray_params& p = *params;
  if (!(p.delta > 0.0f) || !(p.sigma0 > 0.0f) || !(p.eta_minus > 0.0f && p.eta_minus < 1.0f) ||
      !(p.eta_plus >= 1.0f) || !(p.safety > 0.0f && p.safety <= 1.0f) || p.max_iters <= 0 ||
      !isfinite(p.delta) || !isfinite(p.sigma0) || !isfinite(p.eta_plus))
    return SPK_E_INVAL;
  if (p.flags & ~(uint32_t)SPK_FLAG_NO_ROUNDING_BOUND) return SPK_E_INVAL;
  // the boxes take the rays' arithmetic
  if ((box_opts->flags & SPK_FLAG_NO_ROUNDING_BOUND) != (p.flags & SPK_FLAG_NO_ROUNDING_BOUND)) return SPK_E_INVAL;
  if (cam->width <= 0 || cam->height <= 0 || cam->width > 16384 || cam->height > 16384) return SPK_E_INVAL;
  if (tiles_x < 1 || tiles_y < 1 || tiles_x > cam->width || tiles_y > cam->height) return SPK_E_INVAL;
  if (!(cam->tan_x > 0.0f) || !(cam->tan_y > 0.0f) || !isfinite(cam->tan_x) || !isfinite(cam->tan_y))
    return SPK_E_INVAL;
  FrRound R = {};
  const float* vin[4] = {cam->eye, cam->forward, cam->right, cam->up};
  double* vout[4] = {R.cam.eye, R.cam.F, R.cam.Rt, R.cam.U};
  for (int v = 0; v < 4; ++v)
    for (int d = 0; d < 3; ++d) {
      if (!isfinite(vin[v][d])) return SPK_E_INVAL;
      vout[v][d] = (double)vin[v][d];
    }
  // the box construction takes forward, right, up as an orthonormal frame
  const double* fr[3] = {R.cam.F, R.cam.Rt, R.cam.U};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double dot = fr[a][0] * fr[b][0] + fr[a][1] * fr[b][1] + fr[a][2] * fr[b][2];
      if (fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-6) return SPK_E_INVAL;
    }
  if (t_hit == nullptr) return SPK_E_INVAL;
  R.cam.tan_x = cam->tan_x;
  R.cam.tan_y = cam->tan_y;
  R.cam.width = cam->width;
  R.cam.height = cam->height;
  R.p = p;
  const double dist = sqrt(R.cam.eye[0] * R.cam.eye[0] + R.cam.eye[1] * R.cam.eye[1] + R.cam.eye[2] * R.cam.eye[2]);
  // the domain [-1,1]^3 lies in the ball of radius sqrt(3)
  R.t0 = (float)fmax(0.0, dist - 1.7320508075688772 - 1e-6);
  R.t_far = dist + 1.7320508075688772 + 1e-6;
  R.sigma0 = p.sigma0;
  R.t_hit = t_hit;
  R.iters = iters;
  const int64_t npix = (int64_t)cam->width * cam->height;
  const int64_t n0 = (int64_t)tiles_x * tiles_y;
  R.cap = npix;

  // the buffer pointers outlive B, whose destructor frees them
  void *cur = nullptr, *next = nullptr, *cen = nullptr, *axs = nullptr, *miss = nullptr, *lo = nullptr, *hi = nullptr,
       *hp = nullptr, *ht = nullptr, *hs = nullptr, *cnt = nullptr, *org = nullptr, *dir = nullptr, *trel = nullptr,
       *itr = nullptr;
  size_t c_cur = 0, c_next = 0, c_cen = 0, c_axs = 0, c_miss = 0, c_lo = 0, c_hi = 0, c_hp = 0, c_ht = 0, c_hs = 0,
         c_cnt = 0, c_org = 0, c_dir = 0, c_trel = 0, c_itr = 0;
  CallBuffers B;
  B.limit = ctx->workspace_limit;
  B.stream = ctx->stream;
  B.peak = &ctx->ws_peak;
#define SPK_FR_ENSURE(ptr, cap, bytes)              \
  do {                                              \
    spk_status e_ = B.ensure(&(ptr), cap, (bytes)); \
    if (e_ != SPK_OK) return e_;                    \
  } while (0)
  SPK_FR_ENSURE(cur, c_cur, (size_t)npix * sizeof(Frustum));
  SPK_FR_ENSURE(next, c_next, (size_t)npix * sizeof(Frustum));
  SPK_FR_ENSURE(hp, c_hp, (size_t)npix * 8);
  SPK_FR_ENSURE(ht, c_ht, (size_t)npix * 4);
  SPK_FR_ENSURE(hs, c_hs, (size_t)npix * 4);
  SPK_FR_ENSURE(cnt, c_cnt, 256);
  R.cur = (Frustum*)cur;
  R.next = (Frustum*)next;
  R.hand_pix = (int64_t*)hp;
  R.hand_t = (float*)ht;
  R.hand_steps = (int32_t*)hs;
  R.counts = (unsigned long long*)cnt;
  st = launch_fr_zero(R.counts, 3, ctx->stream);
  if (st != SPK_OK) return st;
  st = launch_fr_init(R, tiles_x, tiles_y, ctx->stream);
  if (st != SPK_OK) return st;
  int64_t m = n0, total_steps = 0;
  int32_t rounds = 0;
  unsigned long long hc[3] = {0ull, 0ull, 0ull};
  while (m > 0) {
    if (++rounds > 1000000) return SPK_E_DEVICE;   // not reached: every round makes progress
    SPK_FR_ENSURE(cen, c_cen, (size_t)m * 12);
    SPK_FR_ENSURE(axs, c_axs, (size_t)m * 36);
    SPK_FR_ENSURE(miss, c_miss, (size_t)m);
    SPK_FR_ENSURE(lo, c_lo, (size_t)m * 4);
    SPK_FR_ENSURE(hi, c_hi, (size_t)m * 4);
    R.center = (float*)cen;
    R.axes = (float*)axs;
    R.miss = (uint8_t*)miss;
    R.lo = (const float*)lo;
    R.hi = (const float*)hi;
    st = launch_fr_box(R, m, ctx->stream);
    if (st != SPK_OK) return st;
    BoundJob job = {};
    job.n = m;
    job.mode = IN_GENERAL;
    job.s = 3;
    job.policy = box_opts->policy;
    job.k = box_opts->k;
    job.prec = box_opts->prec;
    job.rigorous = (p.flags & SPK_FLAG_NO_ROUNDING_BOUND) ? 0 : 1;
    job.a = (const float*)cen;
    job.b = (const float*)axs;
    job.lo = (float*)lo;
    job.hi = (float*)hi;
    st = launch_bound(net, job, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    st = launch_fr_update(R, m, ctx->stream);
    if (st != SPK_OK) return st;
    total_steps += m;
    if (hipMemcpyAsync(hc, R.counts, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return SPK_E_DEVICE;
    m = (int64_t)hc[0];
    if (m > npix || (int64_t)hc[1] > npix) return SPK_E_DEVICE;   // disjoint pixel sets: cannot happen
    std::swap(R.cur, R.next);
  }
  const int64_t nh = (int64_t)hc[1];
  if (nh > 0) {
    SPK_FR_ENSURE(org, c_org, (size_t)nh * 12);
    SPK_FR_ENSURE(dir, c_dir, (size_t)nh * 12);
    SPK_FR_ENSURE(trel, c_trel, (size_t)nh * 4);
    SPK_FR_ENSURE(itr, c_itr, (size_t)nh * 4);
    st = launch_fr_rays(R, nh, (float*)org, (float*)dir, ctx->stream);
    if (st != SPK_OK) return st;
    spk_ray_params rp = p;
    rp.clip_to_domain = 1;
    void* counter = nullptr;
    st = ctx_scratch(ctx, 256, &counter);
    if (st != SPK_OK) return st;
    st = launch_rays(net, rp, nh, (const float*)org, (const float*)dir, (float*)trel, (int32_t*)itr,
                     (unsigned long long*)counter, ctx->stream, ctx->num_cus);
    if (st != SPK_OK) return st;
    st = launch_fr_scatter(R, nh, (const float*)trel, (const int32_t*)itr, ctx->stream);
    if (st != SPK_OK) return st;
  }
#undef SPK_FR_ENSURE
  if (stats != nullptr) {
    if (hipMemcpyAsync(hc, R.counts, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess) return SPK_E_DEVICE;
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return SPK_E_DEVICE;
  if (stats != nullptr) {
    stats->frustum_steps = total_steps;
    stats->rays_handed_off = nh;
    stats->ray_iterations = (int64_t)hc[2];
    stats->rounds = rounds;
    stats->reserved = 0;
  }
  return SPK_OK;
}

spk_status spk_eval_points(spk_ctx* ctx, const spk_net* net, int64_t n, const float* x, float* f) {
  if (ctx == nullptr || net == nullptr || n < 0) return SPK_E_INVAL;
  if (n == 0) return SPK_OK;
  if (x == nullptr || f == nullptr) return SPK_E_INVAL;
  const spk_status st = launch_eval(net, n, x, f, ctx->stream, ctx->num_cus);
  if (st == SPK_OK) net_mark_use(net, ctx->stream);
  return st;
}

}  // extern "C"
