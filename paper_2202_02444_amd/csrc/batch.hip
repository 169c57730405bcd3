// Batched range bounds over many networks: one persistent work-queue kernel
// per network class (hidden width, activation, term slots), all of them
// captured once in a HIP graph, so that a single graph launch classifies the
// uneven box frontiers of every network.
//
// Device descriptors per class: the networks' NetDev and BoundJob records
// and the prefix sums of their group counts.  A wavefront takes `chunk`
// consecutive groups from the class counter, finds the network of each group
// by binary search over the prefix sums and runs the same per-group pass as
// the single-network kernel (bound_group.h).  Frontier sizes and buffers may
// change between launches (spk_batch_update rewrites the descriptors); the
// graph stays valid because every kernel drains its queue whatever its size.
#include <algorithm>
#include <new>
#include <utility>
#include <vector>

#include "bound_group.h"

namespace spk {

struct BatchArgs {
  int n_items;
  int chunk;
  const int64_t* prefix;         // [n_items + 1]
  const NetDev* nets;            // [n_items]
  const BoundJob* jobs;          // [n_items]
  unsigned long long* counter;   // work-queue position (groups)
};

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <class S, int ACT, int POL>
__global__ __launch_bounds__(64, 1) void batch_kernel(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) LdsState<S> sm;
  const int lane = threadIdx.x;
  const int64_t total = a.prefix[a.n_items];
  for (;;) {
    unsigned long long got = 0ull;
    if (lane == 0) got = atomicAdd(a.counter, (unsigned long long)a.chunk);
    const int64_t start = uniform64((int64_t)__shfl(got, 0, 64));
    if (start >= total) break;   // every wave reaches this once the queue is drained
    const int64_t end = min(start + (int64_t)a.chunk, total);
    for (int64_t g = start; g < end; ++g) {
      // the network of group g: prefix[lo] <= g < prefix[lo + 1]
      int lo = 0, hi = a.n_items;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.prefix[mid] <= g) lo = mid;
        else hi = mid;
      }
      const NetDev net = a.nets[lo];
      const BoundJob job = a.jobs[lo];
      bound_group<S, ACT, POL>(net, job, sm, g - a.prefix[lo], lane);
    }
  }
}

__global__ void batch_zero_kernel(unsigned long long* counters, int n, int stride) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) counters[(size_t)i * stride] = 0ull;
}

template <class S, int ACT, int POL>
static hipError_t launch_class_k(const BatchArgs& a, int blocks, hipStream_t stream) {
  hipLaunchKernelGGL((batch_kernel<S, ACT, POL>), dim3((unsigned)blocks), dim3(64), 0, stream, a);
  return hipGetLastError();
}

template <int H, int NT, int POL>
static hipError_t launch_class_a(int act, const BatchArgs& a, int blocks, hipStream_t stream) {
  switch (act) {
    case SPK_ACT_RELU: return launch_class_k<Shape<H, NT>, SPK_ACT_RELU, POL>(a, blocks, stream);
    case SPK_ACT_ELU: return launch_class_k<Shape<H, NT>, SPK_ACT_ELU, POL>(a, blocks, stream);
    default: return launch_class_k<Shape<H, NT>, SPK_ACT_SIN, POL>(a, blocks, stream);
  }
}

template <int H>
static hipError_t launch_class_h(int act, int nt, int policy, const BatchArgs& a, int blocks, hipStream_t stream) {
  if (policy == SPK_AFFINE_FIXED) return launch_class_a<H, 1, SPK_AFFINE_FIXED>(act, a, blocks, stream);
  if (nt == 1) return launch_class_a<H, 1, SPK_AFFINE_TRUNCATE>(act, a, blocks, stream);
  return launch_class_a<H, 2, SPK_AFFINE_TRUNCATE>(act, a, blocks, stream);
}

static hipError_t launch_class(int H, int act, int nt, int policy, const BatchArgs& a, int blocks,
                               hipStream_t stream) {
  switch (H) {
    case 32: return launch_class_h<32>(act, nt, policy, a, blocks, stream);
    case 64: return launch_class_h<64>(act, nt, policy, a, blocks, stream);
    case 128: return launch_class_h<128>(act, nt, policy, a, blocks, stream);
    default: return launch_class_h<256>(act, nt, policy, a, blocks, stream);
  }
}

}  // namespace spk

using spk::BatchArgs;

namespace {

constexpr int kCounterStride = 32;   // counters 256 B apart

struct ClassPlan {
  int H = 0, act = 0, nt = 1;
  std::vector<int> items;   // indices into the batch's item list
  int64_t groups = 0;
  int blocks = 0;
  int chunk = 1;
  float tuned_ms = 0.0f;
  size_t off_prefix = 0, off_nets = 0, off_jobs = 0;
};

int bpw_of(int H) { return 256 / H; }

}  // namespace

struct spk_batch {
  int device = 0;
  int num_cus = 0;
  spk_bound_opts opts{};
  std::vector<const spk_net*> nets;
  std::vector<ClassPlan> classes;
  void* dev = nullptr;
  size_t dev_bytes = 0;
  size_t off_counters = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipStream_t> side;   // capture-time fork streams
  std::vector<hipEvent_t> ev;
  bool concurrent = true;          // class kernels as parallel graph branches
  float graph_ms = 0.0f;           // tuned time of one graph launch
  hipEvent_t last = nullptr;       // recorded after every spk_batch_launch
  bool held = false;               // the batch counts as a holder of its networks
  bool frontier = false;           // frontier items: the graph also compacts
  size_t off_compact = 0, off_cprefix = 0;   // CompactItem [n_items], chunk prefix [n_items + 1]
  int compact_blocks = 0;
};

namespace {

BatchArgs class_args(const spk_batch* b, int c) {
  const ClassPlan& p = b->classes[c];
  char* base = (char*)b->dev;
  BatchArgs a;
  a.n_items = (int)p.items.size();
  a.chunk = p.chunk;
  a.prefix = (const int64_t*)(base + p.off_prefix);
  a.nets = (const spk::NetDev*)(base + p.off_nets);
  a.jobs = (const spk::BoundJob*)(base + p.off_jobs);
  a.counter = (unsigned long long*)(base + b->off_counters) + (size_t)c * kCounterStride;
  return a;
}

// Argument checks that read nothing but the item itself.
spk_status valid_item(const spk_batch_item& it) {
  if (it.net == nullptr || it.n < 0) return SPK_E_INVAL;
  if (it.cells == nullptr) {
    if (it.n > 0 && (it.box_lo == nullptr || it.box_hi == nullptr || it.label == nullptr)) return SPK_E_INVAL;
    return SPK_OK;
  }
  const spk_tree_params& t = it.tree;
  if (t.arity != 8) return SPK_E_UNSUPPORTED;
  if (t.max_level < 0 || t.max_level > 20 || it.level < 0 || it.level > t.max_level || t.delta != 0.0f ||
      t.band != 0.0f)
    return SPK_E_INVAL;
  for (int d = 0; d < 3; ++d)
    if (!(t.dom_lo[d] < t.dom_hi[d]) || !isfinite(t.dom_lo[d]) || !isfinite(t.dom_hi[d])) return SPK_E_INVAL;
  if (it.counts == nullptr || it.cap_children < 0 || it.cap_leaves < 0) return SPK_E_INVAL;
  if ((it.cap_children > 0 && it.children == nullptr) || (it.cap_leaves > 0 && it.leaves == nullptr))
    return SPK_E_INVAL;
  if (it.n > 0 && it.label == nullptr) return SPK_E_INVAL;
  return SPK_OK;
}

// Host image of the descriptors (prefix sums, NetDev, BoundJob per class).
spk_status write_descriptors(spk_batch* b, const spk_batch_item* items, hipStream_t stream) {
  std::vector<char> img(b->off_counters, 0);
  for (ClassPlan& p : b->classes) {
    int64_t* prefix = (int64_t*)(img.data() + p.off_prefix);
    spk::NetDev* nd = (spk::NetDev*)(img.data() + p.off_nets);
    spk::BoundJob* jb = (spk::BoundJob*)(img.data() + p.off_jobs);
    prefix[0] = 0;
    for (size_t j = 0; j < p.items.size(); ++j) {
      const spk_batch_item& it = items[p.items[j]];
      nd[j] = it.net->dev;
      spk::BoundJob job = {};
      job.n = it.n;
      job.mode = it.cells ? spk::IN_CELL : spk::IN_AABB;
      job.s = 3;
      job.policy = b->opts.policy;
      job.k = b->opts.k;
      job.rigorous = spk::rigorous_opts(&b->opts) ? 1 : 0;
      job.prec = SPK_PREC_F32;
      job.a = it.box_lo;
      job.b = it.box_hi;
      job.cells = it.cells;
      job.level = it.level;
      for (int d = 0; d < 3; ++d) {
        job.dom_lo[d] = it.tree.dom_lo[d];
        job.dom_hi[d] = it.tree.dom_hi[d];
      }
      job.lo = it.lo;
      job.hi = it.hi;
      job.label = it.label;
      jb[j] = job;
      prefix[j + 1] = prefix[j] + (it.n + bpw_of(p.H) - 1) / bpw_of(p.H);
    }
    p.groups = prefix[p.items.size()];
  }
  if (b->frontier) {
    // the compaction descriptors: one per item in item order, box items empty
    spk::CompactItem* ci = (spk::CompactItem*)(img.data() + b->off_compact);
    int64_t* cp = (int64_t*)(img.data() + b->off_cprefix);
    cp[0] = 0;
    for (size_t i = 0; i < b->nets.size(); ++i) {
      const spk_batch_item& it = items[i];
      spk::CompactItem c = {};
      if (it.cells) {
        c.labels = it.label;
        c.cells = it.cells;
        c.n = it.n;
        c.at_max = it.level == it.tree.max_level ? 1 : 0;
        c.children = it.children;
        c.cap_children = it.cap_children;
        c.leaves = it.leaves;
        c.cap_leaves = it.cap_leaves;
        c.counts = (unsigned long long*)it.counts;
      }
      ci[i] = c;
      cp[i + 1] = cp[i] + (c.n + 63) / 64;
    }
  }
  if (hipMemcpyAsync(b->dev, img.data(), img.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
    return SPK_E_DEVICE;
  // the host image is freed on return: wait for the copy
  return hipStreamSynchronize(stream) == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

void drop_graph(spk_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Capture: zero the counters, then either fork one branch per class
// (independent graph nodes that the runtime may run side by side) and join,
// or chain the class kernels one after another.
spk_status capture(spk_batch* b) {
  drop_graph(b);
  const int nc = (int)b->classes.size();
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SPK_E_DEVICE;
  spk_status st = SPK_OK;
  while ((int)b->side.size() < nc) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) { st = SPK_E_DEVICE; break; }
    b->side.push_back(s);
  }
  while (st == SPK_OK && (int)b->ev.size() < nc + 1) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { st = SPK_E_DEVICE; break; }
    b->ev.push_back(e);
  }
  if (st == SPK_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = SPK_E_DEVICE;
  if (st == SPK_OK) {
    unsigned long long* counters = (unsigned long long*)((char*)b->dev + b->off_counters);
    hipLaunchKernelGGL(spk::batch_zero_kernel, dim3(1), dim3(64), 0, cs, counters, nc, kCounterStride);
    bool ok = hipGetLastError() == hipSuccess && hipEventRecord(b->ev[nc], cs) == hipSuccess;
    for (int c = 0; ok && c < nc; ++c) {
      const ClassPlan& p = b->classes[c];
      if (!b->concurrent) {
        ok = spk::launch_class(p.H, p.act, p.nt, b->opts.policy, class_args(b, c), p.blocks, cs) == hipSuccess;
        continue;
      }
      ok = hipStreamWaitEvent(b->side[c], b->ev[nc], 0) == hipSuccess;
      if (ok) ok = spk::launch_class(p.H, p.act, p.nt, b->opts.policy, class_args(b, c), p.blocks, b->side[c]) ==
                   hipSuccess;
      if (ok) ok = hipEventRecord(b->ev[c], b->side[c]) == hipSuccess;
      if (ok) ok = hipStreamWaitEvent(cs, b->ev[c], 0) == hipSuccess;
    }
    if (ok && b->frontier) {
      // after every class kernel (the join above): compact the frontier items
      const char* base = (const char*)b->dev;
      ok = spk::launch_batch_compact((const spk::CompactItem*)(base + b->off_compact),
                                     (const int64_t*)(base + b->off_cprefix), (int)b->nets.size(), b->compact_blocks,
                                     cs) == hipSuccess;
    }
    hipGraph_t g = nullptr;
    const bool ended = hipStreamEndCapture(cs, &g) == hipSuccess;
    if (!ok || !ended) {
      st = SPK_E_DEVICE;
      if (g) (void)hipGraphDestroy(g);
    } else {
      b->graph = g;
      if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) st = SPK_E_DEVICE;
    }
  }
  (void)hipStreamDestroy(cs);
  if (st != SPK_OK) drop_graph(b);
  return st;
}

// Four persistent workgroups per CU, whatever the class's work at capture
// time: updates may grow the frontiers (a wave that finds the queue empty
// exits at once).
int default_blocks(const spk_batch* b, const ClassPlan& p) {
  (void)p;
  return std::max(b->num_cus * 4, 1);
}

}  // namespace

extern "C" {

spk_status spk_batch_create(spk_ctx* ctx, const spk_bound_opts* opts, int32_t n_items, const spk_batch_item* items,
                            spk_batch** out) {
  if (ctx == nullptr || out == nullptr || n_items <= 0 || items == nullptr) return SPK_E_INVAL;
  spk_status st = spk::valid_opts(opts);
  if (st != SPK_OK) return st;
  if (opts->prec != SPK_PREC_F32) return SPK_E_UNSUPPORTED;   // the class kernels are FP32
  if (opts->policy == SPK_AFFINE_FULL) return SPK_E_UNSUPPORTED;   // no growing generator matrices
  for (int i = 0; i < n_items; ++i) {
    st = valid_item(items[i]);
    if (st != SPK_OK) return st;
  }
  for (int i = 0; i < n_items; ++i)
    if (items[i].net->device != ctx->device) return SPK_E_INVAL;
  spk_batch* b = new (std::nothrow) spk_batch();
  if (b == nullptr) return SPK_E_NOMEM;
  b->device = ctx->device;
  b->num_cus = ctx->num_cus;
  b->opts = *opts;
  const int nt = (opts->policy == SPK_AFFINE_TRUNCATE && opts->k > 15) ? 2 : 1;
  for (int i = 0; i < n_items; ++i) {
    b->nets.push_back(items[i].net);
    const int H = items[i].net->dev.H, act = items[i].net->dev.act;
    int c = -1;
    for (size_t j = 0; j < b->classes.size(); ++j)
      if (b->classes[j].H == H && b->classes[j].act == act) c = (int)j;
    if (c < 0) {
      ClassPlan p;
      p.H = H;
      p.act = act;
      p.nt = nt;
      b->classes.push_back(p);
      c = (int)b->classes.size() - 1;
    }
    b->classes[c].items.push_back(i);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  for (ClassPlan& p : b->classes) {
    p.off_prefix = take(sizeof(int64_t) * (p.items.size() + 1));
    p.off_nets = take(sizeof(spk::NetDev) * p.items.size());
    p.off_jobs = take(sizeof(spk::BoundJob) * p.items.size());
  }
  for (int i = 0; i < n_items; ++i) b->frontier = b->frontier || items[i].cells != nullptr;
  if (b->frontier) {
    b->off_compact = take(sizeof(spk::CompactItem) * (size_t)n_items);
    b->off_cprefix = take(sizeof(int64_t) * ((size_t)n_items + 1));
    b->compact_blocks = ctx->num_cus * 8;
  }
  b->off_counters = off;
  b->dev_bytes = off + sizeof(unsigned long long) * kCounterStride * b->classes.size();
  if (hipMalloc(&b->dev, b->dev_bytes) != hipSuccess) {
    delete b;
    return SPK_E_NOMEM;
  }
  st = write_descriptors(b, items, ctx->stream);
  for (ClassPlan& p : b->classes) p.blocks = default_blocks(b, p);
  if (st == SPK_OK) st = capture(b);
  if (st == SPK_OK && hipEventCreateWithFlags(&b->last, hipEventDisableTiming) != hipSuccess) st = SPK_E_DEVICE;
  if (st != SPK_OK) {
    spk_batch_destroy(b);
    return st;
  }
  for (const spk_net* n : b->nets) n->holders.fetch_add(1);
  b->held = true;
  *out = b;
  return SPK_OK;
}

spk_status spk_batch_update(spk_ctx* ctx, spk_batch* b, int32_t n_items, const spk_batch_item* items) {
  if (ctx == nullptr || b == nullptr || items == nullptr || n_items != (int32_t)b->nets.size()) return SPK_E_INVAL;
  for (int i = 0; i < n_items; ++i) {
    if (items[i].net != b->nets[i]) return SPK_E_INVAL;
    spk_status st = valid_item(items[i]);
    if (st != SPK_OK) return st;
    if (items[i].cells != nullptr && !b->frontier) return SPK_E_INVAL;   // the graph has no compaction
  }
  return write_descriptors(b, items, ctx->stream);
}

spk_status spk_batch_launch(spk_ctx* ctx, spk_batch* b) {
  if (ctx == nullptr || b == nullptr || b->exec == nullptr) return SPK_E_INVAL;
  if (hipGraphLaunch(b->exec, ctx->stream) != hipSuccess) return SPK_E_DEVICE;
  return hipEventRecord(b->last, ctx->stream) == hipSuccess ? SPK_OK : SPK_E_DEVICE;
}

// Launch-shape autotuner: for every class, time each candidate (persistent
// workgroups per CU x groups per queue request) on the current frontiers and
// keep the fastest; then capture the graph again with the winners.
spk_status spk_batch_tune(spk_ctx* ctx, spk_batch* b, int32_t reps) {
  if (ctx == nullptr || b == nullptr || reps <= 0) return SPK_E_INVAL;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SPK_E_DEVICE;
  spk_status st = SPK_OK;
  const int per_cu[] = {1, 2, 4};
  const int chunks[] = {1, 2, 8};
  unsigned long long* counters = (unsigned long long*)((char*)b->dev + b->off_counters);
  for (size_t c = 0; c < b->classes.size() && st == SPK_OK; ++c) {
    ClassPlan& p = b->classes[c];
    if (p.groups == 0) continue;
    float best = -1.0f;
    int best_blocks = p.blocks, best_chunk = p.chunk;
    for (int pc : per_cu) {
      for (int ck : chunks) {
        const int blocks = std::max(1, b->num_cus * pc);   // not capped by the current work: it may grow
        p.chunk = ck;
        BatchArgs a = class_args(b, (int)c);
        float total = 0.0f;
        for (int r = 0; r <= reps && st == SPK_OK; ++r) {   // r = 0 warms up
          hipLaunchKernelGGL(spk::batch_zero_kernel, dim3(1), dim3(64), 0, ctx->stream, counters + c * kCounterStride,
                             1, kCounterStride);
          if (hipEventRecord(e0, ctx->stream) != hipSuccess ||
              spk::launch_class(p.H, p.act, p.nt, b->opts.policy, a, blocks, ctx->stream) != hipSuccess ||
              hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = SPK_E_DEVICE;
            break;
          }
          float ms = 0.0f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (r > 0) total += ms;
        }
        const float avg = total / (float)reps;
        if (st == SPK_OK && (best < 0.0f || avg < best)) {
          best = avg;
          best_blocks = blocks;
          best_chunk = ck;
        }
      }
    }
    p.blocks = best_blocks;
    p.chunk = best_chunk;
    p.tuned_ms = best > 0.0f ? best : 0.0f;
  }
  // whole graph: parallel class branches or a chain, whichever is faster
  float best_graph = -1.0f;
  bool best_conc = true;
  for (int conc = 1; conc >= 0 && st == SPK_OK; --conc) {
    b->concurrent = conc != 0;
    st = capture(b);
    float total = 0.0f;
    for (int r = 0; r <= reps && st == SPK_OK; ++r) {
      if (hipEventRecord(e0, ctx->stream) != hipSuccess || hipGraphLaunch(b->exec, ctx->stream) != hipSuccess ||
          hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = SPK_E_DEVICE;
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) total += ms;
    }
    const float avg = total / (float)reps;
    if (st == SPK_OK && (best_graph < 0.0f || avg < best_graph)) {
      best_graph = avg;
      best_conc = conc != 0;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == SPK_OK) {
    b->concurrent = best_conc;
    b->graph_ms = best_graph;
    st = capture(b);
  }
  return st;
}

spk_status spk_batch_classes(const spk_batch* b, int32_t* n_classes, spk_batch_class* out, int32_t cap) {
  if (b == nullptr || n_classes == nullptr || cap < 0 || (cap > 0 && out == nullptr)) return SPK_E_INVAL;
  *n_classes = (int32_t)b->classes.size();
  for (int32_t c = 0; c < cap && c < *n_classes; ++c) {
    const ClassPlan& p = b->classes[c];
    spk_batch_class& o = out[c];
    o.width = p.H;
    o.act = p.act;
    o.term_slots = 16 * p.nt;
    o.n_nets = (int32_t)p.items.size();
    o.groups = p.groups;
    o.blocks = p.blocks;
    o.chunk = p.chunk;
    o.tuned_ms = p.tuned_ms;
  }
  return SPK_OK;
}

spk_status spk_batch_destroy(spk_batch* b) {
  if (b == nullptr) return SPK_E_INVAL;
  spk_status st = SPK_OK;
  // the device buffers and the graph stay alive until the last launch ended
  if (b->last) {
    if (hipEventSynchronize(b->last) != hipSuccess) st = SPK_E_DEVICE;
    (void)hipEventDestroy(b->last);
  }
  if (b->held)
    for (const spk_net* n : b->nets) n->holders.fetch_sub(1);
  drop_graph(b);
  for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  if (b->dev && hipFree(b->dev) != hipSuccess) st = SPK_E_DEVICE;
  delete b;
  return st;
}

}  // extern "C"
