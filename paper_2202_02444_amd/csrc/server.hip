// Serving loop: continuous batching of box-classify, ray-cast and
// closest-point requests against device-resident networks.
//
// Requests enter a FIFO queue (spk_server_submit never blocks).  A pool of
// worker threads, each owning its own HIP stream and context, admits the
// head request as soon as a worker is free and the bytes of the requests in
// flight plus the head's declared bytes fit the memory budget; admitted
// requests therefore run side by side on separate streams, and requests that
// arrive while others run are admitted as workers and memory free up.  Each
// request runs exactly the calls a standalone caller would make, so its
// result is the same alone and in the mix.  Completions carry the submit,
// start and finish times (steady clock) for latency accounting.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "spk_impl.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Pending {
  spk_request req;
  uint64_t id;
  double submit_s;
};

}  // namespace

struct spk_server {
  std::vector<const spk_net*> nets;
  size_t budget = 0;
  size_t in_flight = 0;
  std::deque<Pending> queue;
  std::deque<spk_completion> done;
  std::mutex mu;
  std::condition_variable cv_work;   // a request was queued, memory freed, or stopping
  std::condition_variable cv_done;   // a request finished
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  int busy = 0;
  bool stop = false;
  uint64_t next_id = 1;
};

namespace {

spk_status run_request(spk_ctx* ctx, const spk_server* s, const spk_request& r) {
  const spk_net* net = s->nets[r.net];
  switch (r.type) {
    case SPK_REQ_CLASSIFY:
      return spk_classify_boxes(ctx, net, &r.opts, r.n, r.a, r.b, (uint8_t*)r.out0, (float*)r.out1,
                                (float*)r.out2, nullptr);
    case SPK_REQ_RAYS:
      return spk_cast_rays(ctx, net, &r.ray, r.n, r.a, r.b, (float*)r.out0, (int32_t*)r.out1);
    case SPK_REQ_CLOSEST:
      return spk_closest_point(ctx, net, &r.opts, &r.tree, r.n, r.a, (float*)r.out0, (float*)r.out1,
                               (float*)r.out2);
  }
  return SPK_E_INVAL;
}

// Bytes of a request's inputs and outputs (device memory the caller owns).
size_t io_bytes(const spk_request& r) {
  const size_t n = (size_t)r.n;
  switch (r.type) {
    case SPK_REQ_CLASSIFY:
      return n * 24 + n + (r.out1 ? n * 4 : 0) + (r.out2 ? n * 4 : 0);
    case SPK_REQ_RAYS:
      return n * 24 + n * 4 + (r.out1 ? n * 4 : 0);
    default:
      return n * 12 + n * 12 + (r.out1 ? n * 4 : 0) + (r.out2 ? n * 4 : 0);
  }
}

void worker_main(spk_server* s, spk_ctx* ctx) {
  for (;;) {
    Pending p;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // FIFO admission: the head runs when its bytes fit beside the requests
      // in flight (a request larger than the whole budget runs alone)
      s->cv_work.wait(lk, [&] {
        if (s->stop) return true;
        if (s->queue.empty()) return false;
        const size_t need = s->queue.front().req.bytes;
        return s->in_flight == 0 || s->in_flight + need <= s->budget;
      });
      if (s->stop) break;
      p = s->queue.front();
      s->queue.pop_front();
      s->in_flight += p.req.bytes;
      ++s->busy;
    }
    const double start = now_s();
    // a closest-point request's workspace stays within its declared bytes
    // beyond its inputs and outputs (box and ray requests use none beyond the
    // context's fixed 4 KiB of scratch)
    const size_t io = io_bytes(p.req);
    ctx->workspace_limit = p.req.type != SPK_REQ_CLOSEST ? 0 : (p.req.bytes > io ? p.req.bytes - io : 1);
    ctx->ws_peak = 0;
    spk_status st = run_request(ctx, s, p.req);
    if (st == SPK_OK) st = spk_ctx_sync(ctx, nullptr);
    const double end = now_s();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->in_flight -= p.req.bytes;
      --s->busy;
      spk_completion c;
      c.id = p.id;
      c.status = st;
      c.type = p.req.type;
      c.n = p.req.n;
      c.submit_s = p.submit_s;
      c.start_s = start;
      c.done_s = end;
      c.workspace_bytes = ctx->ws_peak;
      s->done.push_back(c);
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  spk_ctx_destroy(ctx);
}

}  // namespace

extern "C" {

spk_status spk_server_create(const spk_net* const* nets, int32_t n_nets, size_t mem_budget, int32_t n_workers,
                             spk_server** out) {
  if (nets == nullptr || n_nets <= 0 || n_workers <= 0 || n_workers > 64 || out == nullptr) return SPK_E_INVAL;
  for (int i = 0; i < n_nets; ++i)
    if (nets[i] == nullptr) return SPK_E_INVAL;
  spk_server* s = new (std::nothrow) spk_server();
  if (s == nullptr) return SPK_E_NOMEM;
  s->nets.assign(nets, nets + n_nets);
  s->budget = mem_budget;
  std::vector<spk_ctx*> ctxs;
  for (int w = 0; w < n_workers; ++w) {
    hipStream_t st = nullptr;
    // default-priority streams; the context does not own them, so they are
    // kept and destroyed with the server
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) break;
    spk_ctx* c = nullptr;
    if (spk_ctx_create((void*)st, 0, &c) != SPK_OK) {
      (void)hipStreamDestroy(st);
      break;
    }
    ctxs.push_back(c);
    s->streams.push_back(st);
  }
  if ((int)ctxs.size() != n_workers) {
    for (spk_ctx* c : ctxs) spk_ctx_destroy(c);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return SPK_E_DEVICE;
  }
  for (const spk_net* n : s->nets) n->holders.fetch_add(1);
  for (spk_ctx* c : ctxs) s->workers.emplace_back(worker_main, s, c);
  *out = s;
  return SPK_OK;
}

spk_status spk_server_submit(spk_server* s, const spk_request* req, uint64_t* id) {
  if (s == nullptr || req == nullptr) return SPK_E_INVAL;
  if (req->net < 0 || req->net >= (int32_t)s->nets.size() || req->n < 0) return SPK_E_INVAL;
  if (req->type != SPK_REQ_CLASSIFY && req->type != SPK_REQ_RAYS && req->type != SPK_REQ_CLOSEST)
    return SPK_E_INVAL;
  if (req->n > 0 && (req->a == nullptr || req->out0 == nullptr)) return SPK_E_INVAL;
  if ((req->type == SPK_REQ_CLASSIFY || req->type == SPK_REQ_RAYS) && req->n > 0 && req->b == nullptr)
    return SPK_E_INVAL;
  // affine-full allocates its own workspace per call, outside the admission
  // budget: not served
  if ((req->type == SPK_REQ_CLASSIFY || req->type == SPK_REQ_CLOSEST) && req->opts.policy == SPK_AFFINE_FULL)
    return SPK_E_UNSUPPORTED;
  Pending p;
  p.req = *req;
  p.submit_s = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return SPK_E_BUSY;
    p.id = s->next_id++;
    s->queue.push_back(p);
  }
  if (id) *id = p.id;
  s->cv_work.notify_all();
  return SPK_OK;
}

spk_status spk_server_poll(spk_server* s, spk_completion* out, int32_t max, int32_t* n_done, int32_t wait) {
  if (s == nullptr || n_done == nullptr || max < 0 || (max > 0 && out == nullptr)) return SPK_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (wait && max > 0)
    s->cv_done.wait(lk, [&] { return !s->done.empty() || (s->queue.empty() && s->busy == 0); });
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_done = k;
  return SPK_OK;
}

spk_status spk_server_pending(spk_server* s, int32_t* queued, int32_t* running, size_t* bytes_in_flight) {
  if (s == nullptr) return SPK_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int32_t)s->queue.size();
  if (running) *running = s->busy;
  if (bytes_in_flight) *bytes_in_flight = s->in_flight;
  return SPK_OK;
}

spk_status spk_server_destroy(spk_server* s) {
  if (s == nullptr) return SPK_E_INVAL;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // let admitted and queued requests finish first
    s->cv_done.wait(lk, [&] { return s->queue.empty() && s->busy == 0; });
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->workers) t.join();
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (const spk_net* n : s->nets) n->holders.fetch_sub(1);
  delete s;
  return SPK_OK;
}

}  // extern "C"
