// Continuous-batching server (an extension: the paper runs one
// contraction at a time).
//
// Requests (plan, slice range, host output) are queued by tnc_submit.  A
// request is admitted -- while others are still running -- as soon as a
// slot is free and the arena has room for its planned peak (intermediates of
// its largest chunk, per-chunk base offsets and its FP64 accumulator).
// Every slot owns a worker thread and a HIP stream (default priority), so
// the kernels of admitted requests overlap on the device.  A request's work
// and its chunking depend only on its plan and slice range, so its result is
// the same alone or in a mix.
//
// Overlap helps latency-bound requests (many small launches) and only slows
// compute-bound ones, which already fill the chip alone.  Requests whose
// planned work reaches a threshold are therefore "heavy" and share a lane of
// few slots: a heavy request waits for the heavy ones ahead of it, never for
// light ones, and light requests behind a waiting heavy one go past it.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "serve.hpp"

namespace tnc {

namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) of the context arena.
class ArenaAllocator {
 public:
  explicit ArenaAllocator(int64_t size) { free_[0] = size; }
  int64_t alloc(int64_t bytes) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first;
        const int64_t rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  bool fits(int64_t bytes) const {
    bytes = align_up(bytes);
    for (auto& f : free_)
      if (f.second >= bytes) return true;
    return false;
  }

 private:
  std::map<int64_t, int64_t> free_;
};

struct Request {
  uint64_t id = 0;
  std::shared_ptr<Plan> plan_ref;   // keeps the plan alive while queued or running
  Plan* plan = nullptr;
  int64_t first = 0, count = 0;
  double* out = nullptr;
  int64_t need = 0, work_bytes = 0, acc_off = 0;
  double flops = 0;
  bool heavy = false;       // classified at submission
  bool heavy_slot = false;  // holds a heavy-lane slot while running
  int64_t arena_off = -1;
  Clock::time_point t_submit, t_done;
  bool done = false;
  tnc_status status = TNC_OK;
  std::string err;
};

}  // namespace

struct Server {
  Ctx& ctx;
  int max_inflight;
  size_t queue_cap;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::vector<void*> pinned;            // per slot: pinned result staging
  std::vector<size_t> pinned_bytes;
  ArenaAllocator arena;
  bool stop = false;
  uint64_t next_id = 1;
  int inflight = 0;
  double heavy_flops = 274877906944.0;  // 2^38 planned FLOP
  int heavy_slots = 1;
  int heavy_inflight = 0;

  // Next admissible request (queue order), or end(): heavy requests wait for
  // a heavy slot without blocking light ones; a request that does not fit
  // the free arena blocks everything behind it (no starvation by size).
  std::deque<std::shared_ptr<Request>>::iterator pick() {
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      const Request& r = **it;
      if (r.heavy && heavy_inflight >= heavy_slots) continue;
      return arena.fits(r.need) ? it : queue.end();
    }
    return queue.end();
  }

  Server(Ctx& c, int slots, int cap)
      : ctx(c), max_inflight(slots), queue_cap(cap), arena(static_cast<int64_t>(c.arena_bytes)) {}

  ~Server() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
    }
    cv_work.notify_all();
    for (auto& t : workers) t.join();
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    for (void* p : pinned)
      if (p) (void)hipHostFree(p);
  }

  void start() {
    (void)hipSetDevice(ctx.device);
    for (int i = 0; i < max_inflight; ++i) {
      hipStream_t s = nullptr;
      check_hip(hipStreamCreate(&s), "hipStreamCreate");
      streams.push_back(s);
    }
    pinned.assign(max_inflight, nullptr);
    pinned_bytes.assign(max_inflight, 0);
    for (int i = 0; i < max_inflight; ++i) workers.emplace_back([this, i] { loop(i); });
  }

  void loop(int slot) {
    (void)hipSetDevice(ctx.device);
    hipStream_t stream = streams[slot];
    for (;;) {
      std::shared_ptr<Request> r;
      {
        std::unique_lock<std::mutex> g(mu);
        // drain on stop: keep admitting until the queue is empty
        std::deque<std::shared_ptr<Request>>::iterator it;
        cv_work.wait(g, [&] {
          if (stop && queue.empty()) return true;
          it = pick();
          return it != queue.end();
        });
        if (queue.empty()) return;
        r = *it;
        queue.erase(it);
        r->arena_off = arena.alloc(r->need);
        r->heavy_slot = r->heavy;
        if (r->heavy) ++heavy_inflight;
        ++inflight;
      }
      execute(*r, slot, stream);
      {
        std::lock_guard<std::mutex> g(mu);
        arena.release(r->arena_off, r->need);
        r->t_done = Clock::now();
        r->done = true;
        if (r->heavy_slot) --heavy_inflight;
        --inflight;
      }
      cv_work.notify_all();
      cv_done.notify_all();
    }
  }

  void execute(Request& r, int slot, hipStream_t stream) {
    try {
      Plan& p = *r.plan;
      const ChunkPlan& c0 = *p.chunks[0];
      RunArgs a;
      a.first = r.first;
      a.count = r.count;
      a.arena = ctx.arena + r.arena_off;
      a.arena_bytes = static_cast<size_t>(r.work_bytes);
      a.acc = reinterpret_cast<double2*>(ctx.arena + r.arena_off + r.acc_off);
      a.stream = stream;
      a.fresh_acc = true;
      run_plan(p, a);
      // the slot's pinned staging buffer, grown on demand
      const size_t res_bytes = static_cast<size_t>(c0.R) * 16;
      if (pinned_bytes[slot] < res_bytes) {
        if (pinned[slot]) (void)hipHostFree(pinned[slot]);
        pinned[slot] = nullptr;
        pinned_bytes[slot] = 0;
        check_hip(hipHostMalloc(&pinned[slot], res_bytes, hipHostMallocDefault), "pinned result buffer");
        pinned_bytes[slot] = res_bytes;
      }
      check_hip(hipMemcpyAsync(pinned[slot], a.acc, res_bytes, hipMemcpyDeviceToHost, stream), "result copy");
      check_hip(hipStreamSynchronize(stream), "stream synchronize");
      const double* tmp = static_cast<const double*>(pinned[slot]);
      if (c0.result_perm.empty()) {
        std::memcpy(r.out, tmp, res_bytes);
      } else {
        for (int64_t u = 0; u < c0.R; ++u) {
          r.out[2 * u] = tmp[2 * c0.result_perm[u]];
          r.out[2 * u + 1] = tmp[2 * c0.result_perm[u] + 1];
        }
      }
    } catch (const Error& e) {
      r.status = e.code;
      r.err = e.msg;
    } catch (const std::exception& e) {
      r.status = TNC_E_DEVICE;
      r.err = e.what();
    }
  }
};

std::shared_ptr<Server> make_server(Ctx& ctx, int max_inflight, int queue_cap) {
  auto s = std::make_shared<Server>(ctx, max_inflight, queue_cap);
  s->start();
  return s;
}

}  // namespace tnc

using namespace tnc;

extern "C" {

tnc_status tnc_serve_start(tnc_ctx ctx, int32_t max_inflight, int32_t queue_cap) {
  g_error_clear();
  try {
    if (!ctx) fail(TNC_E_ARG, "ctx is NULL");
    Ctx& c = *ctx->c;
    set_device(c);
    if (!c.arena || !c.arena_bytes) fail(TNC_E_ARG, "serving needs an arena");
    if (max_inflight < 1 || max_inflight > 64 || queue_cap < 1) fail(TNC_E_ARG, "bad serving limits");
    if (c.server) fail(TNC_E_BUSY, "server already running");
    c.server = make_server(c, max_inflight, queue_cap);
  } catch (const Error& e) {
    g_error_set(e.msg);
    return e.code;
  }
  return TNC_OK;
}

tnc_status tnc_serve_set_heavy(tnc_ctx ctx, double heavy_flops, int32_t heavy_slots) {
  g_error_clear();
  if (!ctx || !ctx->c->server || heavy_slots < 1) {
    g_error_set("bad arguments or server not started");
    return TNC_E_ARG;
  }
  Server& s = *ctx->c->server;
  {
    std::lock_guard<std::mutex> g(s.mu);
    s.heavy_flops = heavy_flops;
    s.heavy_slots = heavy_slots;
  }
  s.cv_work.notify_all();
  return TNC_OK;
}

tnc_status tnc_serve_stop(tnc_ctx ctx) {
  g_error_clear();
  if (!ctx) {
    g_error_set("ctx is NULL");
    return TNC_E_ARG;
  }
  ctx->c->server.reset();  // drains the queue: workers finish every request first
  return TNC_OK;
}

tnc_status tnc_submit(tnc_ctx ctx, tnc_plan plan, int64_t first_slice, int64_t n_slices, double* out_c128,
                      tnc_req* id) {
  g_error_clear();
  try {
    if (!ctx || !plan || !out_c128 || !id) fail(TNC_E_ARG, "NULL argument");
    Ctx& c = *ctx->c;
    Server* s = c.server.get();
    if (!s) fail(TNC_E_ARG, "server not started");
    Plan& p = *plan->p;
    if (p.net->ctx != &c) fail(TNC_E_ARG, "plan belongs to another context");
    if (first_slice < 0 || n_slices < 1 || first_slice + n_slices > p.n_slices) fail(TNC_E_ARG, "bad slice range");
    auto r = std::make_shared<Request>();
    r->plan_ref = plan->p;
    r->plan = &p;
    r->first = first_slice;
    r->count = n_slices;
    r->out = out_c128;
    // workspace: intermediates of the largest chunk, chunk base offsets, accumulator
    r->work_bytes = run_workspace_bytes(p, first_slice, n_slices);
    r->acc_off = r->work_bytes;
    r->need = r->work_bytes + align_up(p.chunks[0]->R * 16);
    for (const auto& ch : decompose(p, first_slice, n_slices)) r->flops += p.chunk(ch.first).flops;
    if (r->need > static_cast<int64_t>(c.arena_bytes))
      fail(TNC_E_NOMEM, "request needs " + std::to_string(r->need) + " arena bytes, the arena has " +
                            std::to_string(c.arena_bytes));
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->queue.size() >= s->queue_cap) fail(TNC_E_BUSY, "serving queue full");
      r->heavy = s->heavy_flops > 0 && r->flops >= s->heavy_flops;
      r->id = s->next_id++;
      r->t_submit = Clock::now();
      s->queue.push_back(r);
      s->reqs[r->id] = r;
    }
    s->cv_work.notify_all();
    *id = r->id;
  } catch (const Error& e) {
    g_error_set(e.msg);
    return e.code;
  }
  return TNC_OK;
}

static tnc_status finish(Request& r, double* latency_s) {
  if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
  if (r.status != TNC_OK) g_error_set(r.err);
  return r.status;
}

tnc_status tnc_poll(tnc_ctx ctx, tnc_req id, int32_t* done, double* latency_s) {
  g_error_clear();
  if (!ctx || !done || !ctx->c->server) {
    g_error_set("bad arguments or server not started");
    return TNC_E_ARG;
  }
  Server& s = *ctx->c->server;
  std::lock_guard<std::mutex> g(s.mu);
  auto it = s.reqs.find(id);
  if (it == s.reqs.end()) {
    g_error_set("unknown request id");
    return TNC_E_ARG;
  }
  *done = it->second->done ? 1 : 0;
  if (!it->second->done) {
    if (latency_s) *latency_s = 0;
    return TNC_OK;
  }
  return finish(*it->second, latency_s);
}

tnc_status tnc_wait(tnc_ctx ctx, tnc_req id, double* latency_s) {
  g_error_clear();
  if (!ctx || !ctx->c->server) {
    g_error_set("bad arguments or server not started");
    return TNC_E_ARG;
  }
  Server& s = *ctx->c->server;
  std::unique_lock<std::mutex> g(s.mu);
  auto it = s.reqs.find(id);
  if (it == s.reqs.end()) {
    g_error_set("unknown request id");
    return TNC_E_ARG;
  }
  std::shared_ptr<Request> r = it->second;
  s.cv_done.wait(g, [&] { return r->done; });
  s.reqs.erase(id);
  return finish(*r, latency_s);
}

}  // extern "C"
