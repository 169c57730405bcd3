// Internal definitions shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <utility>
#include <vector>

#include "spk.h"

namespace spk {

// Device copy of a network (uploaded once by spk_net_create).
//
// Layer 0 (3 -> H) is applied on VALU; hidden layers 1..L-2 (H -> H) on MFMA
// (generators, FP32) with the center column on VALU in FP64; the output layer
// (H -> 1) on VALU.  For sine networks each hidden pre-activation is scaled
// by omega0 (Table 2 constant multiplication) before sin.
struct NetDev {
  int L;             // number of linear layers (>= 2)
  int H;             // hidden width
  int act;           // spk_act
  float omega0;      // sine frequency (1 for other activations)
  float cK;          // relative rounding bound of an FP32 H-term dot product (+ bias), any order
  float cD;          // the same for an FP64 H-term dot product
  float c3;          // FP32 3-term dot product (layer 0 generators)
  float eL;          // cK * |b_out| + absolute slack, rounded up
  float bL;          // output bias
  const float* W0;   // [H][4]: layer-0 rows padded to 4 floats
  const float* b0;   // [H]
  const float* Wp;   // (L-2) hidden layers, each H*H floats in MFMA A-fragment order
  const float* bh;   // (L-2) * H biases
  const float* ebh;  // (L-2) * H : cK * |b| + absolute slack, rounded up
  const float* wL;   // [H] output weights
  const uint32_t* Wb;  // (L-2) hidden layers as split BF16 (hi, lo) in 16x16x32 MFMA A-operand order
  float cKs;          // relative rounding bound of a split-BF16 H-term dot product (SPK_PREC_BF16X3)
  const uint32_t* Wh; // (L-2) hidden layers as scaled split FP16, same fragment order as Wb
  const float* wsh;   // (L-2) per-layer unscale factors 2^-sW of Wh
  const float* dwt;   // (L-2) * H : absolute split-FP16 error per unit column scale, per row, rounded up
  float cKh;          // relative rounding bound of a scaled split-FP16 H-term dot product (SPK_PREC_F16X3)
  const float* Wr;    // (L-2) hidden layers in 4x4 blocks [k/4][row/4][row%4][k%4]
};

// Input of a bound launch: which box source feeds the first layer.
enum InputMode { IN_AABB = 0, IN_GENERAL = 1, IN_CELL = 2 };

struct BoundJob {
  int64_t n;
  int mode;           // InputMode
  int s;              // number of box axes (1..3)
  int policy;         // spk_policy (fixed or truncate)
  int k;              // kept terms (truncate)
  int rigorous;       // 1: every rounding bounded (default); 0: the paper's arithmetic + tolerance margin
  int prec;           // spk_prec of the generator products
  // IN_AABB: a = lo [n][3], b = hi [n][3]; IN_GENERAL: a = center [n][3], b = axes [n][s][3]
  const float* a;
  const float* b;
  // IN_CELL
  const uint64_t* cells;
  int level;
  float dom_lo[3];
  float dom_hi[3];
  // outputs (each nullable)
  float* lo;
  float* hi;
  uint8_t* label;
  float* center;
  float* radius;
  float* err;
  int16_t* slot_src;
  unsigned long long* nonfinite;   // device status: boxes with non-finite inputs (nullable)
  float band;         // classification threshold r >= 0: POSITIVE lo > r, NEGATIVE hi < -r
};

// FP32 bounds of the octree cell with Morton code `code` at `level` (bit b of
// the x index at bit 3b, y at 3b+1, z at 3b+2) over the domain box.
__device__ __forceinline__ void cell_box(uint64_t code, int level, const float (&dom_lo)[3],
                                         const float (&dom_hi)[3], float (&lo)[3], float (&hi)[3]) {
  uint32_t idx[3] = {0u, 0u, 0u};
  for (int bb = 0; bb < level; ++bb) {
#pragma unroll
    for (int d = 0; d < 3; ++d) idx[d] |= (uint32_t)((code >> (3 * bb + d)) & 1ull) << bb;
  }
  const float scale = 1.0f / (float)(1u << level);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float size = (dom_hi[d] - dom_lo[d]) * scale;
    lo[d] = dom_lo[d] + (float)idx[d] * size;
    hi[d] = dom_lo[d] + (float)(idx[d] + 1u) * size;
  }
}

// The 6 face centers of a cell (the cell center with one coordinate moved to
// a face), as 18 floats; the closest-point rounds, their seeding descent and
// the convergence test of the frontier rounds share it, so a cell's spanning
// test is the same everywhere.
__device__ __forceinline__ void write_faces(const float (&lo)[3], const float (&hi)[3], float* out) {
  float c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) c[d] = 0.5f * (lo[d] + hi[d]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int d = 0; d < 3; ++d) out[(2 * a + sd) * 3 + d] = (d == a) ? (sd ? hi[d] : lo[d]) : c[d];
}

// Whether six face values show both signs.
__device__ __forceinline__ bool spans6(const float* v) {
  bool neg = false, pos = false;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    neg = neg || v[p] < 0.0f;
    pos = pos || v[p] > 0.0f;
  }
  return neg && pos;
}

struct CellDom {
  float lo[3], hi[3];
};

// Internal label of a frontier cell that passed the convergence test.
constexpr uint8_t kConverged = 3;

// One round of the closest-point search (closest.hip): the frontier of
// (query, cell) pairs at `level` and its outputs.
struct CpLevel {
  int64_t m;                 // frontier items
  int level;
  int at_max;                // 1: no children
  int shared;                // 1: label and fvals already gathered from the distinct cells
  float dom_lo[3];
  float dom_hi[3];
  const uint64_t* codes;     // [m] cells
  const uint32_t* qidx;      // [m] query of each cell
  const uint8_t* label;      // [m] classification of each cell
  const float* q;            // [n][3] queries
  unsigned* best;            // [n] distance bounds (float bits)
  float* point;              // [n][3] candidates
  float* fpts;               // [6m][3] face centers
  float* fvals;              // [6m] f at the face centers
  uint64_t* ncodes;          // [cap] next frontier
  uint32_t* nqidx;           // [cap]
  unsigned long long* ncount;
  int64_t cap;
};

// Greedy descent that seeds the closest-point bound before the level rounds
// (closest.hip): one current cell per query, its 8 children per level.
struct CpDive {
  int64_t n;                 // queries
  int level;                 // level of the children
  float dom_lo[3];
  float dom_hi[3];
  const float* q;            // [n][3] queries
  uint64_t* cur;             // [n] current cell (one level up); all ones: stopped
  uint64_t* codes;           // [8n] children
  const uint8_t* label;      // [8n] classification of the children
  float* fpts;               // [48n][3] face centers of the children
  const float* fvals;        // [48n] f at the face centers
  unsigned* best;            // [n] distance bounds (float bits)
  float* point;              // [n][3] candidates
};

// Sampling in leaf cells (samples.hip).
struct SampleJob {
  const uint64_t* leaves;
  int64_t n_leaves;
  int32_t level;
  int32_t pad;
  float dom_lo[3], dom_hi[3];
  uint64_t seed;
  float band;                // accept |f| < band
  float* points;             // [cap][3] accepted points
  float* f;                  // [cap] nullable
  int64_t cap;
  unsigned long long* counts;   // [0] accepted, [1] accepted with f < 0
};

// Mesh extraction in leaf cells (mesh.hip).
struct MeshJob {
  const uint64_t* leaves;    // [n] Morton codes at `level`
  int32_t level, dense;      // leaf level, dense levels below it
  float dom_lo[3];
  float h[3];                // finest grid spacing
  float* tris;               // [cap][3][3]
  int32_t* src;              // [cap][2] nullable: leaf index, cube index
  int64_t cap;
  unsigned long long* count;
};

// One round of the two-shape intersection test (intersect.hip).
struct IxRound {
  int64_t n;
  int32_t at_max;
  int32_t pad;
  const uint64_t* cells;     // [n] frontier
  const uint8_t* lab_f;      // [n] classification by f
  const uint8_t* lab_g;      // [n] classification by g
  uint64_t* children;        // [cap]
  int64_t cap;
  unsigned long long* counts;   // [4]
};

// Empty-sphere rounds (spheres.hip).
struct EsRound {
  int64_t n;
  const float* p;            // [n][3] query points
  float r0, r_min;
  int64_t* cur;              // [m] live queries of the round
  float* r_cur;              // [m] their radii
  const uint8_t* lab_cur;    // [m] labels of their cubes
  int64_t* next;             // [n] next round
  float* r_next;
  unsigned long long* count;   // next round's size
  float* box_lo;             // [m][3]
  float* box_hi;
  float* radius;             // [n] outputs
  uint8_t* label;
};

// One network's frontier round inside the batched graph (tree.hip).
struct CompactItem {
  const uint8_t* labels;
  const uint64_t* cells;
  int64_t n;                 // 0 for box items
  int32_t at_max;
  int32_t pad;
  uint64_t* children;
  int64_t cap_children;
  uint64_t* leaves;
  int64_t cap_leaves;
  unsigned long long* counts;   // nullable (box items)
};

// Frustum ray casting (frustum.hip).
struct Frustum {
  int32_t x0, x1, y0, y1;   // pixel rectangle [x0, x1) x [y0, y1)
  float t, sigma;
  int32_t steps;            // bound steps taken by the frustum and its ancestors
  int32_t pad;
};

struct FrCam {
  double eye[3], F[3], Rt[3], U[3];   // camera frame (forward, right, up)
  double tan_x, tan_y;
  int32_t width, height;
};

struct FrRound {
  FrCam cam;
  spk_ray_params p;
  float t0, sigma0;
  double t_far;
  Frustum* cur;              // [m] live frusta
  Frustum* next;             // [cap] next round
  int64_t cap;               // width * height
  float* center;             // [m][3] boxes
  float* axes;               // [m][3][3]
  uint8_t* miss;             // [m] box misses the domain
  const float* lo;           // [m] bound of f over the box
  const float* hi;
  int64_t* hand_pix;         // [cap] handed-off pixels
  float* hand_t;
  int32_t* hand_steps;
  unsigned long long* counts;   // [0] next frusta, [1] handed-off pixels, [2] ray iterations
  float* t_hit;              // [height * width]
  int32_t* iters;            // nullable
};

}  // namespace spk

struct spk_net {
  spk::NetDev dev;
  void* dev_block;   // single device allocation holding every array of dev
  int device;
  int32_t n_linear;
  int32_t width;
  // batches and servers that reference the network
  mutable std::atomic<int> holders{0};
  // the last launch on the network per stream (spk_net_destroy checks them)
  mutable std::mutex use_mu;
  mutable std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

struct spk_ctx {
  hipStream_t stream;
  size_t workspace_limit;
  int device;
  int num_cus;
  // scratch (grown on demand)
  void* scratch;
  size_t scratch_bytes;
  // device status word (spk_device_status layout), cleared by spk_ctx_sync
  void* status;
  // largest per-call workspace of the closest-point calls since it was reset
  size_t ws_peak;
};

namespace spk {
// Validation of the bound options shared by every entry point.
inline bool rigorous_opts(const spk_bound_opts* o) { return (o->flags & SPK_FLAG_NO_ROUNDING_BOUND) == 0; }

inline spk_status valid_opts(const spk_bound_opts* o) {
  if (o == nullptr) return SPK_E_INVAL;
  if (o->prec != SPK_PREC_F32 && o->prec != SPK_PREC_BF16X3 && o->prec != SPK_PREC_F16X3 && o->prec != SPK_PREC_F64)
    return SPK_E_UNSUPPORTED;
  if (o->policy != SPK_AFFINE_FIXED && o->policy != SPK_AFFINE_TRUNCATE && o->policy != SPK_AFFINE_FULL)
    return SPK_E_INVAL;
  // affine-full: FP32 generator products only
  if (o->policy == SPK_AFFINE_FULL && o->prec != SPK_PREC_F32) return SPK_E_UNSUPPORTED;
  if (o->policy == SPK_AFFINE_TRUNCATE && (o->k < 3 || o->k > 31)) return SPK_E_UNSUPPORTED;
  if (o->flags & ~(uint32_t)(SPK_FLAG_RIGOROUS | SPK_FLAG_NO_ROUNDING_BOUND)) return SPK_E_INVAL;
  if (o->flags & SPK_FLAG_NO_ROUNDING_BOUND) {
    if ((o->flags & SPK_FLAG_RIGOROUS) || o->prec == SPK_PREC_BF16X3 || o->prec == SPK_PREC_F16X3) return SPK_E_INVAL;
  }
  return SPK_OK;
}

// Records that work on `net` was enqueued on `stream` (for SPK_E_BUSY).
void net_mark_use(const spk_net* net, hipStream_t stream);

// Launch helpers implemented in bound.hip / tree.hip / rays.hip.
spk_status launch_bound(const spk_net* net, const BoundJob& job, hipStream_t stream, int num_cus);
// affine-full (full.hip): hidden width 256, FP32 products; allocates its
// workspace stream-ordered for the launch
spk_status launch_full(const spk_net* net, const BoundJob& job, hipStream_t stream, int num_cus);
spk_status launch_compact(const uint8_t* labels, const uint64_t* cells, int64_t n, bool at_max,
                          uint64_t* children, int64_t cap_children, uint64_t* leaves, int64_t cap_leaves,
                          int64_t* counts, void* status, hipStream_t stream, int num_cus);
spk_status launch_eval(const spk_net* net, int64_t n, const float* x, float* f, hipStream_t stream,
                       int num_cus);
spk_status launch_rays(const spk_net* net, const spk_ray_params& p, int64_t n, const float* origin,
                       const float* dir, float* t_hit, int32_t* iters, unsigned long long* counter,
                       hipStream_t stream, int num_cus);
spk_status launch_cp_init(int64_t n, uint64_t* codes, uint32_t* qidx, unsigned* best, float* point,
                          hipStream_t stream, int num_cus);
spk_status launch_cp_round(const spk_net* net, const CpLevel& L, hipStream_t stream, int num_cus);
// Distinct cells of a round: temporary bytes for m codes; sort + unique into
// ucodes with the count in *nu (device); then, for the distinct cells U (U.m
// of them, classified into ulabel), the face values and the gather into every
// item's label and fvals.
size_t cp_dedup_temp_bytes(int64_t m);
spk_status launch_cp_dedup(const uint64_t* codes, uint64_t* sorted, uint64_t* ucodes, int64_t* nu, int64_t m,
                           int level, void* temp, size_t temp_bytes, hipStream_t stream);
spk_status launch_cp_shared(const spk_net* net, const CpLevel& U, const uint64_t* codes, int64_t m,
                            const uint8_t* ulabel, float* ufvals, uint8_t* label, float* fvals, hipStream_t stream,
                            int num_cus);
// The batched graph's compaction: zero every item's counts, then compact the
// labelled cells of every item (one launch each).
hipError_t launch_batch_compact(const CompactItem* items, const int64_t* prefix, int n_items, int blocks,
                                hipStream_t stream);
// The convergence test of a frontier round: face centers of every cell,
// their f, and UNKNOWN cells that span the level set relabelled kConverged.
spk_status launch_converge(const spk_net* net, uint8_t* labels, const uint64_t* cells, int64_t n, int level,
                           const float (&dom_lo)[3], const float (&dom_hi)[3], float* fpts, float* fvals,
                           hipStream_t stream, int num_cus);
spk_status launch_sample_chunk(const spk_net* net, const SampleJob& J, int64_t i0, int64_t m, float* pts, float* vals,
                               hipStream_t stream, int num_cus);
spk_status launch_mesh_chunk(const spk_net* net, const MeshJob& M, int64_t l0, int64_t nl, float* pts, float* vals,
                             hipStream_t stream, int num_cus);
spk_status launch_ix_round(const IxRound& X, hipStream_t stream, int num_cus);
spk_status launch_es_init(const EsRound& E, hipStream_t stream);
spk_status launch_es_boxes(const EsRound& E, int64_t m, hipStream_t stream);
spk_status launch_es_update(const EsRound& E, int64_t m, hipStream_t stream);
spk_status launch_fr_init(const FrRound& R, int tiles_x, int tiles_y, hipStream_t stream);
spk_status launch_fr_box(const FrRound& R, int64_t m, hipStream_t stream);
spk_status launch_fr_update(const FrRound& R, int64_t m, hipStream_t stream);
spk_status launch_fr_zero(unsigned long long* counts, int n, hipStream_t stream);
spk_status launch_fr_rays(const FrRound& R, int64_t n, float* origin, float* dir, hipStream_t stream);
spk_status launch_fr_scatter(const FrRound& R, int64_t n, const float* trel, const int32_t* itr, hipStream_t stream);
spk_status launch_cp_dive_init(int64_t n, uint64_t* cur, hipStream_t stream, int num_cus);
spk_status launch_cp_dive_children(const CpDive& D, hipStream_t stream, int num_cus);
spk_status launch_cp_dive_pick(const CpDive& D, hipStream_t stream, int num_cus);
spk_status launch_cp_finish(int64_t n, const float* q, const unsigned* best, float* point, float* dist,
                            float* best_out, hipStream_t stream, int num_cus);
}  // namespace spk
