/*
 * spk.h -- C ABI of the MI355X range-analysis library.
 *
 * Guaranteed range bounds of an MLP implicit function f: R^3 -> R over many
 * boxes, rays and cells at once, after Sharp & Jacobson, "Spelunking the Deep:
 * Guaranteed Queries on General Neural Implicit Surfaces via Range Analysis"
 * (ACM TOG 41(4), 2022):
 *
 *   spk_range_bound        RangeBound, Procedure 1, steps 1-3 (the bound)
 *   spk_classify_boxes     RangeBound, Procedure 1, steps 1-6 (sign class)
 *   spk_subdivide_frontier one parallel round of BuildSpatialTree,
 *                          Procedure 3 / Section 4.5 (fixed depth, Section 4.7)
 *   spk_cast_rays          CastRay, Procedure 2 (with the Appendix B step safety)
 *
 * Conventions shared by every call
 *  - Every call returns an spk_status.  Nothing aborts or prints.
 *  - Pointers documented "dev" are device (HBM) pointers allocated and owned by
 *    the caller; "host" pointers are read during the call only.
 *  - All work is enqueued asynchronously on the context's HIP stream.  The
 *    returned status covers argument validation and launch errors; call
 *    spk_ctx_sync to wait.  Arguments are validated before any HIP call.
 *  - An spk_net is read-only after creation and may be shared by contexts.
 *    One spk_ctx must not be used from two host threads at once.
 *  - n == 0 is a no-op returning SPK_OK.
 *  - Bounds (default): the returned [lo, hi] is a provably sound enclosure of
 *    f over the box.  The affine-arithmetic bound of the paper is evaluated
 *    with generators in FP32 on MFMA, center and linearisation parameters in
 *    FP64, and every rounding bounded a priori and folded into the condensed
 *    term (a per-neuron error symbol, Appendix A), so the form encloses the
 *    exact network at every layer.  With SPK_FLAG_NO_ROUNDING_BOUND the
 *    arithmetic is the paper's, which ignores rounding (Section 3.4): the raw
 *    bound matches the exact affine arithmetic to about 1e-6 relative and
 *    [lo, hi] adds a tolerance margin of 2^-18 (|center| + radius), which is
 *    not a proof.  Non-finite inputs give lo = -inf, hi = +inf and label
 *    UNKNOWN.
 */
#ifndef SPK_H
#define SPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPK_OK = 0,
  SPK_E_INVAL = 1,        /* bad argument (null pointer, bad size or enum)        */
  SPK_E_NOMEM = 2,        /* device or host allocation failed                     */
  SPK_E_NOSPC = 3,        /* an output array is too small; see the call           */
  SPK_E_DEVICE = 4,       /* a HIP runtime call failed                            */
  SPK_E_UNSUPPORTED = 5,  /* valid request the library does not implement        */
  SPK_E_BUSY = 6,         /* object still in use                                  */
  SPK_E_LIMIT = 7         /* request exceeds a fixed capacity of the library       */
} spk_status;

/* Activations (Table 3).  SPK_ACT_SIN is sin(omega0 * z) (SIREN convention). */
typedef enum { SPK_ACT_RELU = 0, SPK_ACT_ELU = 1, SPK_ACT_SIN = 2 } spk_act;

/* Condensation policies (Section 3.3).
 *  SPK_AFFINE_FIXED     every new term goes into the condensed term.
 *  SPK_AFFINE_TRUNCATE  the k largest terms are kept (3 <= k <= 31).
 *  SPK_AFFINE_FULL      every term is kept: the generator matrix grows by the
 *                       hidden width at each activation.  Hidden width 128 or
 *                       256 and SPK_PREC_F32 only (else SPK_E_UNSUPPORTED);
 *                       each call allocates, stream-ordered on the context's
 *                       stream, a workspace of min(n, 4 x CUs) x H x
 *                       (32 + H (L-2)) floats (L linear layers; 1.9 GB for
 *                       H = 256 and 8 hidden layers on 256 CUs), SPK_E_NOMEM
 *                       if that fails.  The rounding-
 *                       bounded mode puts every rounding into the new term of
 *                       its neuron.  Not available to spk_batch_create,
 *                       spk_subdivide_frontier_noalloc or the server
 *                       (SPK_E_UNSUPPORTED). */
typedef enum { SPK_AFFINE_FIXED = 0, SPK_AFFINE_TRUNCATE = 1, SPK_AFFINE_FULL = 2 } spk_policy;

/* Arithmetic of the generator products Y = W X of the hidden layers.
 *  SPK_PREC_F32    FP32 MFMA (16x16x4), FP32 accumulation.
 *  SPK_PREC_BF16X3 split BF16: W = W_hi + W_lo and X = X_hi + X_lo (round to
 *                  nearest BF16 each), W_hi X_hi + W_hi X_lo + W_lo X_hi on the
 *                  BF16 MFMA (16x16x32) with FP32 accumulation.  The dropped
 *                  W_lo X_lo and split residuals are bounded a priori like
 *                  every other rounding (SPK_FLAG_NO_ROUNDING_BOUND is
 *                  rejected).  Hidden width 256 only (else
 *                  SPK_E_UNSUPPORTED); single-network bound calls only.
 *  SPK_PREC_F16X3  split FP16 with power-of-two scaling: each hidden layer's W
 *                  is scaled by 2^sW (max |W| 2^sW in [2^14, 2^15)) and each
 *                  generator column of X by 2^sc (its max in [2^14, 2^15)),
 *                  hi = RNE16(v), lo = RNE16((v - hi) 2^11); W_hi X_hi and
 *                  2^-11 (W_hi X_lo + W_lo X_hi) on the FP16 MFMA (16x16x32)
 *                  with FP32 accumulation, then unscaled.  The rigorous
 *                  radius bounds the dropped lo*lo term, the W split
 *                  residual (measured exactly at network creation), the X
 *                  split residual, FP16 underflow and the accumulation.
 *                  Same restrictions as SPK_PREC_BF16X3.
 *  SPK_PREC_F64    generator products on the FP64 MFMA (16x16x4, W and X
 *                  widened exactly from FP32), FP64 accumulation, the center
 *                  column in FP64 through the same MFMA; results stored in
 *                  FP32.  With the rounding bound this keeps the enclosure
 *                  close to the exact affine bound also on the smallest boxes
 *                  of deep networks, at about twice the matrix-core time of
 *                  FP32.  Hidden width 256 only (else SPK_E_UNSUPPORTED);
 *                  single-network bound calls only. */
typedef enum { SPK_PREC_F32 = 0, SPK_PREC_BF16X3 = 1, SPK_PREC_F16X3 = 2, SPK_PREC_F64 = 3 } spk_prec;

/* uint8 sign classes of Procedure 1. */
enum { SPK_UNKNOWN = 0, SPK_POSITIVE = 1, SPK_NEGATIVE = 2 };

/* spk_bound_opts.flags */
enum {
  /* the rounding-error bound (the default; accepted for explicitness) */
  SPK_FLAG_RIGOROUS = 1u,
  /* the paper's arithmetic without the rounding-error bound, widened by the
     tolerance margin only (for comparison with the exact arithmetic); not
     combinable with SPK_FLAG_RIGOROUS or the split precisions */
  SPK_FLAG_NO_ROUNDING_BOUND = 2u
};

typedef struct {
  int32_t policy;   /* spk_policy                                                */
  int32_t k;        /* affine-truncate: number of kept terms, 3 <= k <= 31       */
  int32_t prec;     /* spk_prec                                                  */
  uint32_t flags;   /* SPK_FLAG_* bits                                           */
} spk_bound_opts;

typedef struct spk_net spk_net;
typedef struct spk_ctx spk_ctx;

const char* spk_status_str(spk_status s);

/* Library version string. */
const char* spk_version(void);

/*
 * spk_net_create: upload an MLP (Section 2 setting): n_linear linear layers,
 * the activation after every layer but the last.
 *   widths  host [n_linear+1]: widths[0] = 3, widths[n_linear] = 1, all hidden
 *           widths equal to one H in {32, 64, 128, 256}; n_linear in [2, 16].
 *   W       host [n_linear] pointers, W[l] row-major [widths[l+1]][widths[l]].
 *   b       host [n_linear] pointers, b[l] of length widths[l+1].
 *   act     spk_act; omega0 the sine frequency (ignored unless SPK_ACT_SIN, > 0).
 * The library copies everything into its own device buffers (on the current
 * HIP device), precomputes the per-layer rounding constants in FP64 and owns
 * the result until spk_net_destroy.  Returns SPK_E_UNSUPPORTED for shapes
 * outside the list above.
 */
spk_status spk_net_create(int32_t n_linear, const int32_t* widths, const float* const* W,
                          const float* const* b, int32_t act, float omega0, spk_net** out);
/* Frees the network.  SPK_E_BUSY (nothing freed) while a batch or a server
 * still references it, or while work launched on it by a bound, frontier,
 * ray, closest-point or evaluation call has not finished on its stream (the
 * non-allocating frontier call and calls made under HIP graph capture are
 * not tracked: the caller orders those). */
spk_status spk_net_destroy(spk_net* net);

/*
 * spk_ctx_create: a context bound to one HIP stream (a hipStream_t passed as
 * void*; NULL is the default stream).  workspace_bytes is an upper bound on the
 * scratch memory the context may allocate (0 = no limit).
 */
spk_status spk_ctx_create(void* stream, size_t workspace_bytes, spk_ctx** out);
spk_status spk_ctx_destroy(spk_ctx* ctx);

/* Device-side conditions of the context's calls since the previous
 * spk_ctx_sync (the kernels write them; spk_ctx_sync reads and clears them). */
typedef struct {
  int64_t nonfinite_inputs;  /* boxes whose input coordinates were not all finite
                                (their results are [-inf, +inf], UNKNOWN)       */
  int32_t nospc;             /* 1: a frontier round found more children or
                                leaves than its capacity                        */
  int32_t reserved;
  int64_t need_children;     /* largest required capacities among those rounds  */
  int64_t need_leaves;
} spk_device_status;

/* Wait for all work of the context's stream and read the device status word.
 * status (host, nullable) receives it.  Returns SPK_E_NOSPC when a frontier
 * round overflowed a capacity since the previous sync (the counts of that
 * round hold its required sizes), else the stream's status. */
spk_status spk_ctx_sync(spk_ctx* ctx, spk_device_status* status);

/*
 * Optional diagnostic outputs of the bound calls (all dev, nullable).
 *   center, radius  [n]: the bound's center and radius before the last
 *                   widening.  Under SPK_FLAG_NO_ROUNDING_BOUND these are the
 *                   paper's arithmetic (lo_raw = center - radius, hi_raw =
 *                   center + radius); by default the radius already holds the
 *                   folded rounding bounds of every layer.
 *   err             [n]: the widening applied beyond center -/+ radius: the
 *                   rounding of the output layer itself (default), else the
 *                   tolerance margin.
 *   slot_src        [n_linear-1][n][32] int16: for affine-truncate, after
 *                   each activation (n_linear-1 of them) and for each of the
 *                   32 term slots of each box: -1 the slot kept its previous
 *                   term, j >= 0 it now holds the new term of neuron j, -2 the
 *                   slot is empty.  Slot 0 is the center (always -1).
 */
typedef struct {
  float* center;
  float* radius;
  float* err;
  int16_t* slot_src;
} spk_bound_aux;

/*
 * spk_range_bound: Procedure 1, steps 1-3 for general boxes.
 *   n       number of boxes; s in {1, 2, 3} box axes per box.
 *   center  dev [n][3]; axes dev [n][s][3] (half-axis vectors, need not be
 *           axis-aligned; the box is center + sum_i eps_i axes[i], |eps_i| <= 1).
 *   lo, hi  dev [n] outputs: a sound enclosure of f over each box.
 *   aux     nullable, see spk_bound_aux.
 */
spk_status spk_range_bound(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts, int64_t n,
                           int32_t s, const float* center, const float* axes, float* lo, float* hi,
                           const spk_bound_aux* aux);

/*
 * spk_classify_boxes: Procedure 1 for axis-aligned boxes [box_lo, box_hi]
 * (dev [n][3] each).  label dev [n] (uint8 SPK_UNKNOWN/POSITIVE/NEGATIVE:
 * POSITIVE iff lo > 0, NEGATIVE iff hi < 0).  lo, hi dev [n] nullable.
 */
spk_status spk_classify_boxes(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts, int64_t n,
                              const float* box_lo, const float* box_hi, uint8_t* label, float* lo,
                              float* hi, const spk_bound_aux* aux);

/* Tree parameters: the domain box and the fixed maximum octree level.
 * delta > 0 turns on the convergence test of Procedure 3 for small cells
 * (spk_subdivide_frontier only; the other calls require 0): at a level whose
 * cells' widest side is below delta / sqrt(3), an UNKNOWN cell whose six face
 * centers show both signs of f (FP32 evaluation) is within delta of the level
 * set and final; it goes to `leaves` instead of splitting.
 * band r > 0 (spk_subdivide_frontier only; not with delta) classifies
 * against the band |f| <= r instead of the level set (Section 4.6): a cell is
 * POSITIVE when f > r on it and NEGATIVE when f < -r, so the UNKNOWN cells
 * cover every point with |f| <= r. */
typedef struct {
  float dom_lo[3];
  float dom_hi[3];
  int32_t max_level;   /* 0 <= max_level <= 20                                   */
  int32_t arity;       /* 8 (octree); other values give SPK_E_UNSUPPORTED        */
  float delta;         /* 0: fixed depth; > 0: convergence test (finite)         */
  float band;          /* 0: the level set; > 0: the band |f| <= band (finite)   */
} spk_tree_params;

/*
 * spk_subdivide_frontier: one parallel round of Procedure 3 at fixed depth.
 * cells dev [n] are Morton codes at `level` (bit b of the x index at bit 3b,
 * y at 3b+1, z at 3b+2).  Each cell is classified; POSITIVE and NEGATIVE cells
 * are counted; UNKNOWN cells with level < max_level write their 8 children
 * (code << 3 | octant) to `children`; UNKNOWN cells at max_level are copied to
 * `leaves` (the cells handed to mesh extraction, Section 4.7), and so are the
 * converged cells of the delta test (tree->delta > 0; not available in
 * spk_subdivide_frontier_noalloc, SPK_E_UNSUPPORTED).
 *   children dev [cap_children], leaves dev [cap_leaves] (either may be NULL
 *            when its capacity is 0).
 *   counts   dev int64 [4]: n_children, n_leaves, n_pos, n_neg.  The call sets
 *            them (it does not accumulate).  Output order is unspecified.
 * When a capacity is too small the required count is still written to
 * `counts`, entries beyond the capacity are dropped, and the next
 * spk_ctx_sync returns SPK_E_NOSPC with the required sizes in its status.
 */
spk_status spk_subdivide_frontier(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                                  const spk_tree_params* tree, int32_t level, const uint64_t* cells,
                                  int64_t n, uint64_t* children, int64_t cap_children, uint64_t* leaves,
                                  int64_t cap_leaves, int64_t* counts);

/*
 * spk_subdivide_frontier_noalloc: spk_subdivide_frontier for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors, but the per-cell labels of the round live in a fixed, library-owned
 * device array of SPK_NOALLOC_MAX_CELLS bytes (one copy per GPU, held until
 * the process ends) instead of the context's workspace, and the call makes no
 * allocation (no hipMalloc / hipFree).
 *   n > SPK_NOALLOC_MAX_CELLS returns SPK_E_LIMIT before any HIP call.
 * Every call on one GPU shares that array: calls that overlap on a GPU (from
 * several contexts or streams) race and must be serialised by the caller.
 * The array needs no clearing: each call writes every label it reads.
 */
#define SPK_NOALLOC_MAX_CELLS 16777216
spk_status spk_subdivide_frontier_noalloc(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                                          const spk_tree_params* tree, int32_t level, const uint64_t* cells,
                                          int64_t n, uint64_t* children, int64_t cap_children, uint64_t* leaves,
                                          int64_t cap_leaves, int64_t* counts);

/* CastRay parameters (Procedure 2; Section 4.1 delta; Appendix B safety). */
typedef struct {
  float delta;          /* convergence length, e.g. 1e-3                            */
  float t_max;          /* miss distance when clip_to_domain == 0                   */
  float sigma0;         /* initial step, e.g. t_max / 10                            */
  float eta_minus;      /* step shrink factor, e.g. 0.5                             */
  float eta_plus;       /* step growth factor, e.g. 1.5                             */
  float safety;         /* accepted step fraction, e.g. 0.98                        */
  int32_t max_iters;    /* per-ray iteration cap (> 0)                              */
  int32_t clip_to_domain; /* 1: march each ray over its chord of [-1,1]^3 only     */
  uint32_t flags;       /* 0: every segment bound carries its rounding bound, so a
                           step is accepted only when the exact network has no
                           root on the segment; SPK_FLAG_NO_ROUNDING_BOUND: the
                           paper's arithmetic with the tolerance margin          */
} spk_ray_params;

/*
 * spk_sample_leaves (surface sampling, Section 4.6; bulk properties,
 * Section 4.8): n_samples uniform points in the union of n_leaves leaf cells
 * of one level (e.g. the UNKNOWN leaves of a tree built with
 * spk_tree_params.band = r, which cover every point with |f| <= r).  Sample
 * i takes outputs 4i .. 4i+3 of the splitmix64 generator seeded with `seed`
 * (z = seed + (k + 1) 0x9e3779b97f4a7c15; z = (z ^ z >> 30) 0xbf58476d1ce4e5b9;
 * z = (z ^ z >> 27) 0x94d049bb133111eb; z ^ z >> 31): leaf = output 4i mod
 * n_leaves, offsets u_d = (output 4i+1+d >> 40) 2^-24, point = lo + u (hi - lo)
 * (FP32).  Samples with |f| < band (band = +inf: all) are written, in
 * unspecified order, to points dev [cap][3] and f dev [cap] (nullable).
 *   n_accepted host: accepted samples (SPK_E_NOSPC when above cap; the first
 *              cap are written); n_below host nullable: accepted with f < 0.
 *   points = NULL (cap 0): only the counts are computed.
 * Synchronous; 16 bytes per sample of a chunk of at most 2^24 samples,
 * stream-ordered within the context's workspace limit.
 */
spk_status spk_sample_leaves(spk_ctx* ctx, const spk_net* net, const spk_tree_params* tree, int32_t level,
                             int64_t n_leaves, const uint64_t* leaves, int64_t n_samples, uint64_t seed, float band,
                             float* points, float* f, int64_t cap, int64_t* n_accepted, int64_t* n_below);

/*
 * spk_mesh_leaves (Section 4.7): triangles of the level set inside leaf cells
 * (Morton codes at `level` in tree's domain, e.g. the leaves of the last
 * frontier round).  Each leaf is sampled on the grid of dense_levels (0..4)
 * further subdivisions (Appendix B evaluates the lowest levels densely; its
 * meshes use 3): points dom_lo + g h with g the index on the finest grid, so
 * neighbouring leaves share their face samples exactly, and every grid cube
 * is meshed by marching cubes without a case table (each face joins its
 * crossing edges; a face with four crossings cuts off the corners whose sign
 * differs from the mean of its four values; the loops are triangulated as
 * fans; edge points interpolate f linearly; f > 0 is outside).
 *   tris    dev float [cap_tris][3][3]; tri_src dev int32 [cap_tris][2]
 *           nullable: the leaf's index and the cube's index in it
 *           (x fastest).  Output order is unspecified.
 *   n_tris  host: the number of triangles; SPK_E_NOSPC when it exceeds
 *           cap_tris (the first cap_tris are written).
 * Synchronous; about 12 bytes per grid point of a chunk of leaves (at most
 * 256 MiB) stream-ordered within the context's workspace limit.
 */
spk_status spk_mesh_leaves(spk_ctx* ctx, const spk_net* net, const spk_tree_params* tree, int32_t level,
                           int32_t dense_levels, int64_t n_leaves, const uint64_t* leaves, float* tris,
                           int32_t* tri_src, int64_t cap_tris, int64_t* n_tris);

/*
 * spk_intersect (Section 4.9): whether the solids {f < 0} and {g < 0} of two
 * networks overlap inside the tree domain, by octree rounds (arity 8) that
 * bound both networks on every frontier cell: a cell with either function
 * POSITIVE cannot hold a common point and is dropped; a cell with both
 * NEGATIVE lies inside both solids and ends the search (witness: the
 * smallest Morton code among such cells of that level); other cells split
 * until tree->max_level, where they remain undecided.  Synchronous; the
 * frontier buffers (74 bytes per cell) are stream-ordered within the
 * context's workspace limit (SPK_E_NOMEM beyond it).
 */
enum { SPK_NO_INTERSECTION = 0, SPK_INTERSECTION = 1, SPK_INTERSECTION_UNDECIDED = 2 };
typedef struct {
  int32_t result;           /* SPK_NO_INTERSECTION / SPK_INTERSECTION / _UNDECIDED */
  int32_t level;            /* witness level (SPK_INTERSECTION), else -1          */
  uint64_t cell;            /* witness Morton code                                */
  int64_t undecided;        /* cells left at max_level (_UNDECIDED)               */
  int64_t cells_bounded;    /* cell bounds evaluated (both networks)              */
  int32_t rounds;
  int32_t reserved;
} spk_intersect_result;

spk_status spk_intersect(spk_ctx* ctx, const spk_net* net_f, const spk_net* net_g, const spk_bound_opts* opts,
                         const spk_tree_params* tree, spk_intersect_result* out);

/*
 * spk_empty_spheres (Section 4.4): for each point p_i (dev [n][3]) the first
 * radius r in r0, r0/2, r0/4, ... with r >= r_min such that the bound
 * classifies the cube [p - r, p + r]^3 (rounded outwards) as POSITIVE or
 * NEGATIVE, so that the ball of radius r around p holds no point of the level
 * set.  radius dev [n]: that r, 0 if none; label dev uint8 [n]: the cube's
 * class (UNKNOWN with radius 0).  Synchronous (one host round trip per
 * halving); buffers about 45 bytes per point, stream-ordered within the
 * context's workspace limit.  0 < r_min <= r0 (finite), else SPK_E_INVAL.
 */
spk_status spk_empty_spheres(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts, int64_t n, const float* p,
                             float r0, float r_min, float* radius, uint8_t* label);

/*
 * Frustum ray casting (Section 4.3; Appendix B).  A pinhole camera: pixel
 * (px, py), row-major from the top row, looks from eye along
 * normalize(forward + x right + y up) with
 *   x = (2 (px + 0.5) / width - 1) tan_x,  y = (1 - 2 (py + 0.5) / height) tan_y.
 * forward, right, up must be orthonormal (dot products within 1e-6).
 */
typedef struct {
  float eye[3];
  float forward[3];
  float right[3];
  float up[3];
  float tan_x, tan_y;   /* tangents of the half fields of view (> 0)            */
  int32_t width, height;
} spk_camera;

typedef struct {
  int64_t frustum_steps;     /* frustum boxes bounded                           */
  int64_t rays_handed_off;   /* pixels continued as single rays                 */
  int64_t ray_iterations;    /* Procedure 2 iterations of those rays            */
  int32_t rounds;            /* frustum rounds                                  */
  int32_t reserved;
} spk_frustum_stats;

/*
 * spk_cast_frusta: cast the camera's width x height pixel rays against the
 * level set inside the domain [-1,1]^3 by marching a tiles_x x tiles_y grid
 * of coarse frusta (pixel rectangles) forward.  Each step bounds f over the
 * oriented camera-frame box of the frustum between distances t and t + sigma
 * (extended to the rays' spherical front); the step is taken (t += safety
 * sigma, sigma *= eta_plus) when the box misses the domain or f is bounded
 * away from zero on it, else sigma *= eta_minus, and a frustum whose width at
 * t + sigma exceeds 2 sigma (or with sigma < delta) splits in half along its
 * wider image direction.  A single-pixel frustum continues as Procedure 2
 * from its t over the ray's chord of the domain.  Frusta start at the
 * distance of the domain's bounding sphere.
 *   params   delta, sigma0, eta_minus, eta_plus, safety, max_iters (of the
 *            per-pixel rays) and flags as in spk_cast_rays; t_max and
 *            clip_to_domain are not used.
 *   box_opts policy, k, prec of the frustum-box bounds; its
 *            SPK_FLAG_NO_ROUNDING_BOUND bit must equal params->flags'.
 *   t_hit    dev [height * width]: distance from the eye along the pixel's
 *            unit ray to its hit, +inf for none.
 *   iters    dev int32 [height * width] nullable: frustum steps the pixel
 *            took part in plus its ray iterations.
 *   stats    host nullable.
 * The call is synchronous (one host round trip per frustum round) and takes
 * its buffers (about 60 bytes per pixel) stream-ordered within the context's
 * workspace limit.
 */
spk_status spk_cast_frusta(spk_ctx* ctx, const spk_net* net, const spk_ray_params* params,
                           const spk_bound_opts* box_opts, const spk_camera* cam, int32_t tiles_x, int32_t tiles_y,
                           float* t_hit, int32_t* iters, spk_frustum_stats* stats);

/*
 * spk_cast_rays: Procedure 2 for n rays (origin, dir dev [n][3]; dir unit
 * length).  Segment bounds use affine-fixed (the paper's ray-casting choice).
 *   t_hit  dev [n]: first t with a sign change within delta, +inf for no hit.
 *   iters  dev int32 [n] nullable: loop iterations per ray.
 */
spk_status spk_cast_rays(spk_ctx* ctx, const spk_net* net, const spk_ray_params* params, int64_t n,
                         const float* origin, const float* dir, float* t_hit, int32_t* iters);

/*
 * spk_closest_point: closest point on the level set f = 0 (Section 4.10) for
 * n query points q dev [n][3] (n < 2^32).  The octree of `tree` is searched
 * down to tree->max_level; cells are classified with `opts` (the paper uses
 * affine-fixed).  A cell spans the level set when it is UNKNOWN and f takes
 * both signs on its six face centers; it then contains a zero of f, so the
 * farthest distance from q to it bounds the distance to the surface.  Result
 * for query i: the center of a spanning cell (reached through UNKNOWN
 * ancestors) minimising that farthest distance.
 *   point  dev [n][3]: the cell center; NaN when no cell spans the surface.
 *   dist   dev [n] nullable: |point - q|, +inf when none.
 *   bound  dev [n] nullable: the farthest distance from q to that cell (an
 *          upper bound of the distance from q to the surface), +inf when none.
 * The call runs one round per level and waits for each round (it returns with
 * the stream synchronized); it allocates its frontier buffers in device
 * memory and frees them before returning.  Queries run in chunks of up to
 * 1024; a chunk whose frontier would exceed the context's workspace limit
 * (16 GiB when the context has none) is retried in halves, and SPK_E_NOMEM
 * is returned only when a single query's frontier does not fit.
 */
spk_status spk_closest_point(spk_ctx* ctx, const spk_net* net, const spk_bound_opts* opts,
                             const spk_tree_params* tree, int64_t n, const float* q, float* point, float* dist,
                             float* bound);

/*
 * Batched bounds over many networks (Procedure 1 for each network's boxes,
 * and for frontier items one Procedure 3 round).  The batch groups its
 * networks into classes (hidden width x activation), runs one persistent
 * work-queue kernel per class and captures all of them once in a HIP graph,
 * followed by one compaction kernel over every frontier item:
 * spk_batch_launch is a single graph launch that classifies every network's
 * boxes or cells and compacts every frontier, however uneven the sizes.
 *
 *   spk_batch_create  items host [n_items] (read during the call); the nets
 *                     must live on the context's device and stay alive
 *                     while the batch exists.  Writes descriptors to device
 *                     memory it owns and captures the graph (synchronizes).
 *   spk_batch_update  same networks in the same order with new box counts
 *                     and buffers (e.g. the next frontier); no re-capture.
 *   spk_batch_launch  enqueue the graph on the context's stream.
 *   spk_batch_tune    autotuner: per class, times every launch shape
 *                     (persistent workgroups 1, 2, 4 per CU x 1, 2, 8 groups
 *                     per queue request) reps times on the current items and
 *                     keeps the fastest; then times the whole graph with the
 *                     class kernels as parallel branches and as a chain, and
 *                     keeps the faster capture.  Runs the kernels, so the
 *                     outputs are written.
 *   spk_batch_classes the class table (n_classes set; up to cap entries).
 */
typedef struct {
  const spk_net* net;
  int64_t n;               /* boxes (or cells) of this network (>= 0)       */
  const float* box_lo;     /* dev [n][3] (box items)                        */
  const float* box_hi;     /* dev [n][3] (box items)                        */
  uint8_t* label;          /* dev [n] uint8 class                           */
  float* lo;               /* dev [n] nullable                              */
  float* hi;               /* dev [n] nullable                              */
  /* Frontier items (Procedure 3 rounds): with cells non-null the n boxes
   * are the Morton cells of `level` in tree (arity 8), and the graph also
   * compacts the round as spk_subdivide_frontier does: UNKNOWN cells below
   * tree.max_level emit their 8 children (at most cap_children written),
   * UNKNOWN cells at max_level go to leaves (at most cap_leaves);
   * counts dev int64 [4] = {children, leaves, positive, negative}, the
   * required sizes when a capacity is exceeded.  A batch created without
   * frontier items takes none later. */
  const uint64_t* cells;   /* dev [n] nullable: a box item                  */
  int32_t level;
  int32_t reserved;
  spk_tree_params tree;
  uint64_t* children;      /* dev [cap_children] nullable if cap is 0       */
  int64_t cap_children;
  uint64_t* leaves;        /* dev [cap_leaves] nullable if cap is 0         */
  int64_t cap_leaves;
  int64_t* counts;         /* dev [4] (frontier items)                      */
} spk_batch_item;

typedef struct spk_batch spk_batch;

typedef struct {
  int32_t width;           /* hidden width H                                */
  int32_t act;             /* spk_act                                       */
  int32_t term_slots;      /* 16 or 32 affine term slots per box            */
  int32_t n_nets;
  int64_t groups;          /* wavefront work items at the last update       */
  int32_t blocks;          /* persistent workgroups of the class kernel     */
  int32_t chunk;           /* groups per work-queue request                 */
  float tuned_ms;          /* best time seen by spk_batch_tune (0: untuned)  */
} spk_batch_class;

spk_status spk_batch_create(spk_ctx* ctx, const spk_bound_opts* opts, int32_t n_items, const spk_batch_item* items,
                            spk_batch** out);
spk_status spk_batch_update(spk_ctx* ctx, spk_batch* batch, int32_t n_items, const spk_batch_item* items);
spk_status spk_batch_launch(spk_ctx* ctx, spk_batch* batch);
spk_status spk_batch_tune(spk_ctx* ctx, spk_batch* batch, int32_t reps);
spk_status spk_batch_classes(const spk_batch* batch, int32_t* n_classes, spk_batch_class* out, int32_t cap);
spk_status spk_batch_destroy(spk_batch* batch);

/*
 * Serving: continuous batching of requests against device-resident networks.
 * A server owns n_workers worker threads, each with its own HIP stream and
 * context.  Requests queue in FIFO order; the head request is admitted as soon
 * as a worker is free and the declared bytes of the requests in flight plus
 * its own fit mem_budget (a request larger than the budget runs alone).
 * Admitted requests run side by side on their streams; each one makes exactly
 * the calls a standalone caller would make, so its result does not depend on
 * the mix.  The server never allocates request buffers: the caller allocates
 * inputs and outputs (device memory) and keeps them alive until the request's
 * completion is returned by spk_server_poll.
 *
 * spk_request fields by type:
 *   SPK_REQ_CLASSIFY  a = box_lo, b = box_hi [n][3]; out0 = label (uint8 [n]),
 *                     out1 = lo, out2 = hi (float [n], nullable); opts.
 *   SPK_REQ_RAYS      a = origin, b = dir [n][3]; out0 = t_hit (float [n]),
 *                     out1 = iters (int32 [n], nullable); ray.
 *   SPK_REQ_CLOSEST   a = query [n][3]; out0 = point [n][3], out1 = dist,
 *                     out2 = bound (float [n], nullable); opts, tree.
 *   bytes             the request's device footprint: its inputs and outputs
 *                     plus the library workspace it may use.  Admission keeps
 *                     the bytes of the requests in flight within the budget,
 *                     and the library keeps a request's workspace within
 *                     bytes minus the sizes of its inputs and outputs (closest
 *                     point shrinks its query chunks to fit; SPK_E_NOMEM when
 *                     one query's frontier does not fit).  Beyond that the
 *                     workers hold only their contexts' few hundred bytes of
 *                     scratch and status.  Requests with SPK_AFFINE_FULL are
 *                     refused (SPK_E_UNSUPPORTED at submit): that policy
 *                     allocates its workspace outside the budget.
 * spk_server_poll returns up to max completions (wait != 0: block until one is
 * available or nothing is queued or running).  spk_server_destroy waits for
 * every queued and running request, then stops the workers.
 */
typedef enum { SPK_REQ_CLASSIFY = 0, SPK_REQ_RAYS = 1, SPK_REQ_CLOSEST = 2 } spk_req_type;

typedef struct {
  int32_t type;              /* spk_req_type                                   */
  int32_t net;               /* index into the server's network list           */
  int64_t n;
  const float* a;
  const float* b;
  void* out0;
  void* out1;
  void* out2;
  size_t bytes;
  spk_bound_opts opts;
  spk_ray_params ray;
  spk_tree_params tree;
} spk_request;

typedef struct {
  uint64_t id;
  int32_t status;            /* spk_status of the request                      */
  int32_t type;
  int64_t n;
  double submit_s, start_s, done_s;   /* steady-clock seconds                  */
  uint64_t workspace_bytes;  /* largest library workspace the request held      */
} spk_completion;

typedef struct spk_server spk_server;

spk_status spk_server_create(const spk_net* const* nets, int32_t n_nets, size_t mem_budget, int32_t n_workers,
                             spk_server** out);
spk_status spk_server_submit(spk_server* server, const spk_request* req, uint64_t* id);
spk_status spk_server_poll(spk_server* server, spk_completion* out, int32_t max, int32_t* n_done, int32_t wait);
spk_status spk_server_pending(spk_server* server, int32_t* queued, int32_t* running, size_t* bytes_in_flight);
spk_status spk_server_destroy(spk_server* server);

/* Point evaluation f(x) for x dev [n][3] -> f dev [n] (FP32). */
spk_status spk_eval_points(spk_ctx* ctx, const spk_net* net, int64_t n, const float* x, float* f);

#ifdef __cplusplus
}
#endif

#endif /* SPK_H */
