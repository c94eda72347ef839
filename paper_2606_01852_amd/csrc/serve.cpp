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
//
// Row requests of a batcher (a plan with a batch label whose rows come from
// the requests) are taken together: up to B queued rows of one batcher form
// one job, whose rows are written into the batch-labelled leaves before the
// plan runs once, so the same-shape steps of those requests share each
// launch.  A batcher runs one job at a time (its leaves hold one batch).
//
// Light requests whose plans have one structure (the same network shape,
// path, slicing, precision, chunking and tile variants: e.g. amplitudes of
// several circuits of one geometry, or slice ranges of one network) are
// fused when they are launch-bound (kFuseFlopsPerLaunch): a worker that
// admits such a request also admits up to fuse_max - 1 queued requests with
// the same structure key, and runs them in lockstep with the launches of
// one run: every MFMA step and every tree level's small GEMMs and gathers
// as one grouped launch over all of them.  Each result is bitwise the one
// the request gets alone.
//
// On a host-only context the server admits and queues exactly as it would
// on a device (admission by planned arena bytes, the heavy lane, batcher
// tokens) but executes nothing: every request completes with
// TNC_E_UNSUPPORTED.  That lets the queueing code run, with its threads,
// where there is no GPU.
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

}  // namespace

struct Request {
  uint64_t id = 0;
  std::shared_ptr<Plan> plan_ref;   // keeps the plan alive while queued or running (dropped when done)
  Plan* plan = nullptr;
  int64_t first = 0, count = 0;
  double* out = nullptr;
  int64_t need = 0, work_bytes = 0, acc_off = 0;
  double flops = 0;
  bool heavy = false;       // classified at submission
  bool heavy_slot = false;  // holds a heavy-lane slot while running
  int64_t arena_off = -1;
  std::shared_ptr<Batcher> batcher;  // row request (or a batcher's token): its batcher
  bool token = false;                // stands for the batcher's waiting rows in the queue
  std::vector<float2> row;           // row values of the listed leaves (complex64)
  std::string key;                   // structure key (fusable light request), or empty
  LockstepInfo tables;               // its share of a fused job's tables
  int64_t table_off = -1, table_bytes = 0;  // a fused job's table (first request of the job)
  Clock::time_point t_submit, t_done;
  bool done = false;
  tnc_status status = TNC_OK;
  std::string err;
};

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
  std::vector<void*> pinned_in;         // per slot: pinned staging of batch rows
  std::vector<size_t> pinned_in_bytes;
  std::vector<void*> pinned_tab;        // per slot: pinned staging of grouped-launch tables
  std::vector<size_t> pinned_tab_bytes;
  int fuse_max = 8;                     // requests per fused job (1: no fusion)
  // A light request is fused only below this many planned FLOP per launch
  // of its own run.  Fusing shares launches; it pays while a run waits on
  // them, and costs the overlap of separate streams once a run's own
  // arithmetic fills the GPU.  Measured on 8 slots (random grid circuits,
  // 512 requests): 2.3x the unfused rate at 1.4e7 FLOP per launch (4x5,
  // depth 10), 1.05x at 4.5e8 (5x5, depth 10), 0.96x at 4.1e9 (5x6, depth
  // 10); the default, 2^30, lies between the last two.
  double fuse_flops_per_launch = 1073741824.0;
  int64_t n_jobs = 0, n_fused_jobs = 0, n_fused_requests = 0;
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
    {
      std::lock_guard<std::recursive_mutex> rt(runtime_mu());
      for (hipStream_t s : streams)
        if (s) (void)hipStreamDestroy(s);
    }
    for (void* p : pinned) pinned_free(p);
    for (void* p : pinned_in) pinned_free(p);
    for (void* p : pinned_tab) pinned_free(p);
  }

  void start() {
    if (!ctx.host_only) {
      (void)hipSetDevice(ctx.device);
      std::lock_guard<std::recursive_mutex> rt(runtime_mu());
      for (int i = 0; i < max_inflight; ++i) {
        hipStream_t s = nullptr;
        check_hip(hipStreamCreate(&s), "hipStreamCreate");
        streams.push_back(s);
      }
    } else {
      streams.assign(max_inflight, nullptr);
    }
    pinned.assign(max_inflight, nullptr);
    pinned_bytes.assign(max_inflight, 0);
    pinned_in.assign(max_inflight, nullptr);
    pinned_in_bytes.assign(max_inflight, 0);
    pinned_tab.assign(max_inflight, nullptr);
    pinned_tab_bytes.assign(max_inflight, 0);
    for (int i = 0; i < max_inflight; ++i) workers.emplace_back([this, i] { loop(i); });
  }

  void loop(int slot) {
    if (!ctx.host_only) (void)hipSetDevice(ctx.device);
    hipStream_t stream = streams[slot];
    for (;;) {
      std::vector<std::shared_ptr<Request>> job;  // one request, or rows of one batcher
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
        if ((*it)->token) {
          // a batcher's token: up to B of its waiting rows, in submission order
          Batcher& b = *(*it)->batcher;
          while (!b.rows.empty() && static_cast<int64_t>(job.size()) < b.B) {
            job.push_back(b.rows.front());
            b.rows.pop_front();
          }
          b.queued = false;
          queue.erase(it);
          if (job.empty()) continue;  // no rows behind the token (never queued so)
          b.busy = true;
          job[0]->heavy = b.flops >= heavy_flops && heavy_flops > 0;
        } else {
          job.push_back(*it);
          queue.erase(it);
        }
        Request& r = *job[0];
        r.arena_off = arena.alloc(r.need);
        r.heavy_slot = r.heavy;
        if (r.heavy) ++heavy_inflight;
        ++inflight;
        if (!r.key.empty() && fuse_max > 1) gather_fusable(job);
        ++n_jobs;
        if (job.size() > 1) {
          ++n_fused_jobs;
          n_fused_requests += static_cast<int64_t>(job.size());
        }
      }
      if (job[0]->batcher)
        execute_rows(job, slot, stream);
      else if (job.size() > 1)
        execute_fused(job, slot, stream);
      else
        execute(*job[0], slot, stream);
      // plans of finished requests, released at the end of this iteration,
      // after the lock and the notifications (a last reference tears the
      // plan down, with device synchronizations)
      std::vector<std::shared_ptr<Plan>> finished;
      {
        std::lock_guard<std::mutex> g(mu);
        Request& r = *job[0];
        arena.release(r.arena_off, r.need);
        if (!r.batcher)  // a fused job's other requests and its table
          for (size_t q = 1; q < job.size(); ++q) arena.release(job[q]->arena_off, job[q]->need);
        if (r.table_off >= 0) arena.release(r.table_off, r.table_bytes);
        r.table_off = -1;
        if (r.heavy_slot) --heavy_inflight;
        --inflight;
        if (r.batcher) {
          std::shared_ptr<Batcher> b = r.batcher;
          b->busy = false;
          if (!b->rows.empty()) enqueue_token(b);  // rows that came in meanwhile
          // drop the rows' references before they are marked done: with its
          // handle destroyed and no rows left the batcher releases its
          // network here, before any waiter returns
          for (auto& q : job) q->batcher.reset();
        }
        const Clock::time_point now = Clock::now();
        for (auto& q : job) {
          q->t_done = now;
          q->done = true;
          q->row.clear();
          q->row.shrink_to_fit();
          finished.push_back(std::move(q->plan_ref));
          q->plan = nullptr;
        }
      }
      cv_work.notify_all();
      cv_done.notify_all();
    }
  }

  // A fused job (server mutex held): queued light requests with job[0]'s
  // structure key join it while the arena has room for each of them and for
  // the job's grouped-launch table; a request that does not fit stays queued.
  void gather_fusable(std::vector<std::shared_ptr<Request>>& job) {
    Request& r0 = *job[0];
    for (auto it = queue.begin(); it != queue.end() && static_cast<int>(job.size()) < fuse_max;) {
      Request& q = **it;
      if (q.token || q.heavy || q.key != r0.key) {
        ++it;
        continue;
      }
      const int64_t off = arena.alloc(q.need);
      if (off < 0) break;
      q.arena_off = off;
      job.push_back(*it);
      it = queue.erase(it);
    }
    if (job.size() == 1) return;
    r0.table_bytes = static_cast<int64_t>(lockstep_table_bytes(r0.tables, static_cast<int>(job.size())));
    r0.table_off = arena.alloc(r0.table_bytes);
    if (r0.table_off >= 0) return;
    // no room for the table: the others go back to the front of the queue
    for (size_t q = job.size() - 1; q >= 1; --q) {
      arena.release(job[q]->arena_off, job[q]->need);
      job[q]->arena_off = -1;
      queue.push_front(job[q]);
    }
    job.resize(1);
  }

  // Queue a token for a batcher's waiting rows (server mutex held).
  void enqueue_token(const std::shared_ptr<Batcher>& b) {
    auto t = std::make_shared<Request>();
    t->token = true;
    t->batcher = b;
    t->need = b->need;
    t->flops = b->flops;
    t->heavy = heavy_flops > 0 && b->flops >= heavy_flops;
    queue.push_back(t);
    b->queued = true;
  }

  // Grow a slot's pinned staging buffer to `bytes` (only this slot's worker
  // uses it, after its previous job has synchronised).
  static void* staging(std::vector<void*>& bufs, std::vector<size_t>& sizes, int slot, size_t bytes) {
    if (sizes[slot] < bytes) {
      pinned_free(bufs[slot]);
      bufs[slot] = nullptr;
      sizes[slot] = 0;
      bufs[slot] = pinned_alloc(bytes, "pinned staging buffer");
      sizes[slot] = bytes;
    }
    return bufs[slot];
  }

  static constexpr const char* kHostOnly = "host-only context: the request was admitted but nothing runs";

  // Run `plan` over all its slices in the request's arena interval; the FP64
  // result lands in the slot's pinned buffer (synchronous on `stream`).
  const double* run_to_host(Request& r, Plan& p, int slot, hipStream_t stream) {
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
    const size_t res_bytes = static_cast<size_t>(c0.R) * 16;
    void* host = staging(pinned, pinned_bytes, slot, res_bytes);
    check_hip(hipMemcpyAsync(host, a.acc, res_bytes, hipMemcpyDeviceToHost, stream), "result copy");
    check_hip(hipStreamSynchronize(stream), "stream synchronize");
    return static_cast<const double*>(host);
  }

  // Rows of one batcher: rows 0..k-1 of each listed leaf (the batch label is
  // its outermost mode, so they are contiguous) come from the k requests in
  // order, the plan runs once, and request j gets row j of the result.
  void execute_rows(std::vector<std::shared_ptr<Request>>& job, int slot, hipStream_t stream) {
    Request& r0 = *job[0];
    if (ctx.host_only) {
      for (auto& q : job) {
        q->status = TNC_E_UNSUPPORTED;
        q->err = kHostOnly;
      }
      return;
    }
    try {
      Batcher& b = *r0.batcher;
      Plan& p = *b.plan;
      Net& n = *p.net;
      const int64_t k = static_cast<int64_t>(job.size());
      float2* in = static_cast<float2*>(
          staging(pinned_in, pinned_in_bytes, slot, static_cast<size_t>(k * b.row_total) * sizeof(float2)));
      int64_t off = 0, src = 0;
      for (size_t i = 0; i < b.leaves.size(); ++i) {
        const int64_t re = b.row_elems[i];
        for (int64_t j = 0; j < k; ++j)
          std::memcpy(in + off + j * re, job[j]->row.data() + src, static_cast<size_t>(re) * sizeof(float2));
        check_hip(hipMemcpyAsync(n.leaf[b.leaves[i]].ptr, in + off, static_cast<size_t>(k * re) * sizeof(float2),
                                 hipMemcpyHostToDevice, stream),
                  "row upload");
        off += k * re;
        src += re;
      }
      const double* tmp = run_to_host(r0, p, slot, stream);
      const ChunkPlan& c0 = *p.chunks[0];
      for (int64_t j = 0; j < k; ++j) {
        double* out = job[j]->out;
        for (int64_t u = 0; u < b.out_row; ++u) {
          const int64_t g = j * b.out_row + u;
          const int64_t s = c0.result_perm.empty() ? g : c0.result_perm[g];
          out[2 * u] = tmp[2 * s];
          out[2 * u + 1] = tmp[2 * s + 1];
        }
      }
    } catch (const Error& e) {
      for (auto& q : job) {
        q->status = e.code;
        q->err = e.msg;
      }
    } catch (const std::exception& e) {
      for (auto& q : job) {
        q->status = TNC_E_DEVICE;
        q->err = e.what();
      }
    }
  }

  // Requests of one structure in lockstep (run_lockstep), every result
  // staged through the slot's pinned buffer.
  void execute_fused(std::vector<std::shared_ptr<Request>>& job, int slot, hipStream_t stream) {
    if (ctx.host_only) {
      for (auto& q : job) {
        q->status = TNC_E_UNSUPPORTED;
        q->err = kHostOnly;
      }
      return;
    }
    try {
      const int K = static_cast<int>(job.size());
      std::vector<LockstepRun> runs(K);
      size_t res_total = 0;
      for (int q = 0; q < K; ++q) {
        Request& r = *job[q];
        runs[q].plan = r.plan;
        RunArgs& a = runs[q].a;
        a.first = r.first;
        a.count = r.count;
        a.arena = ctx.arena + r.arena_off;
        a.arena_bytes = static_cast<size_t>(r.work_bytes);
        a.acc = reinterpret_cast<double2*>(ctx.arena + r.arena_off + r.acc_off);
        a.stream = stream;
        a.fresh_acc = true;
        res_total += static_cast<size_t>(r.plan->chunks[0]->R) * 16;
      }
      Request& r0 = *job[0];
      void* host_tab = staging(pinned_tab, pinned_tab_bytes, slot, static_cast<size_t>(r0.table_bytes));
      run_lockstep(runs, host_tab, ctx.arena + r0.table_off, static_cast<size_t>(r0.table_bytes), stream);
      char* host = static_cast<char*>(staging(pinned, pinned_bytes, slot, res_total));
      size_t off = 0;
      for (int q = 0; q < K; ++q) {
        const size_t b = static_cast<size_t>(job[q]->plan->chunks[0]->R) * 16;
        check_hip(hipMemcpyAsync(host + off, runs[q].a.acc, b, hipMemcpyDeviceToHost, stream), "result copy");
        off += b;
      }
      check_hip(hipStreamSynchronize(stream), "stream synchronize");
      off = 0;
      for (int q = 0; q < K; ++q) {
        Request& r = *job[q];
        const ChunkPlan& c0 = *r.plan->chunks[0];
        const double* tmp = reinterpret_cast<const double*>(host + off);
        if (c0.result_perm.empty()) {
          std::memcpy(r.out, tmp, static_cast<size_t>(c0.R) * 16);
        } else {
          for (int64_t u = 0; u < c0.R; ++u) {
            r.out[2 * u] = tmp[2 * c0.result_perm[u]];
            r.out[2 * u + 1] = tmp[2 * c0.result_perm[u] + 1];
          }
        }
        off += static_cast<size_t>(c0.R) * 16;
      }
    } catch (const Error& e) {
      for (auto& q : job) {
        q->status = e.code;
        q->err = e.msg;
      }
    } catch (const std::exception& e) {
      for (auto& q : job) {
        q->status = TNC_E_DEVICE;
        q->err = e.what();
      }
    }
  }

  void execute(Request& r, int slot, hipStream_t stream) {
    if (ctx.host_only) {
      r.status = TNC_E_UNSUPPORTED;
      r.err = kHostOnly;
      return;
    }
    try {
      Plan& p = *r.plan;
      const ChunkPlan& c0 = *p.chunks[0];
      const double* tmp = run_to_host(r, p, slot, stream);
      if (c0.result_perm.empty()) {
        std::memcpy(r.out, tmp, static_cast<size_t>(c0.R) * 16);
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

Batcher::~Batcher() {
  if (plan) --plan->net->n_batchers;
}

std::shared_ptr<Server> make_server(Ctx& ctx, int max_inflight, int queue_cap) {
  auto s = std::make_shared<Server>(ctx, max_inflight, queue_cap);
  s->start();
  return s;
}

}  // namespace tnc

using namespace tnc;

extern "C" {

tnc_status tnc_serve_start(tnc_ctx ctx, int32_t max_inflight, int32_t queue_cap) {
  TNC_TRY
    if (!ctx) fail(TNC_E_ARG, "ctx is NULL");
    Ctx& c = *ctx->c;
    if (!c.host_only) {
      set_device(c);
      if (!c.arena) fail(TNC_E_ARG, "serving needs an arena");
    }
    if (!c.arena_bytes) fail(TNC_E_ARG, "serving needs an arena size");
    if (max_inflight < 1 || max_inflight > 64 || queue_cap < 1) fail(TNC_E_ARG, "bad serving limits");
    if (c.server) fail(TNC_E_BUSY, "server already running");
    c.server = make_server(c, max_inflight, queue_cap);
  TNC_CATCH
}

tnc_status tnc_serve_set_heavy(tnc_ctx ctx, double heavy_flops, int32_t heavy_slots) {
  TNC_TRY
  if (!ctx || !ctx->c->server || heavy_slots < 1) fail(TNC_E_ARG, "bad arguments or server not started");
  Server& s = *ctx->c->server;
  {
    std::lock_guard<std::mutex> g(s.mu);
    s.heavy_flops = heavy_flops;
    s.heavy_slots = heavy_slots;
  }
  s.cv_work.notify_all();
  TNC_CATCH
}

tnc_status tnc_serve_set_fusion(tnc_ctx ctx, int32_t max_requests, double flops_per_launch) {
  TNC_TRY
  if (!ctx || !ctx->c->server || max_requests < 1 || max_requests > 64 || !(flops_per_launch > 0))
    fail(TNC_E_ARG, "bad arguments or server not started");
  Server& s = *ctx->c->server;
  std::lock_guard<std::mutex> g(s.mu);
  s.fuse_max = max_requests;
  s.fuse_flops_per_launch = flops_per_launch;
  TNC_CATCH
}

tnc_status tnc_serve_get_stats(tnc_ctx ctx, int64_t* jobs, int64_t* fused_jobs, int64_t* fused_requests) {
  TNC_TRY
  if (!ctx || !ctx->c->server || !jobs || !fused_jobs || !fused_requests)
    fail(TNC_E_ARG, "bad arguments or server not started");
  Server& s = *ctx->c->server;
  std::lock_guard<std::mutex> g(s.mu);
  *jobs = s.n_jobs;
  *fused_jobs = s.n_fused_jobs;
  *fused_requests = s.n_fused_requests;
  TNC_CATCH
}

tnc_status tnc_serve_stop(tnc_ctx ctx) {
  TNC_TRY
  if (!ctx) fail(TNC_E_ARG, "ctx is NULL");
  ctx->c->server.reset();  // drains the queue: workers finish every request first
  TNC_CATCH
}

tnc_status tnc_submit(tnc_ctx ctx, tnc_plan plan, int64_t first_slice, int64_t n_slices, double* out_c128,
                      tnc_req* id) {
  TNC_TRY
    if (!ctx || !plan || !out_c128 || !id) fail(TNC_E_ARG, "NULL argument");
    Ctx& c = *ctx->c;
    Server* s = c.server.get();
    if (!s) fail(TNC_E_ARG, "server not started");
    Plan& p = *plan->p;
    if (p.net->ctx != &c) fail(TNC_E_ARG, "plan belongs to another context");
    if (p.net->n_batchers.load() > 0)
      fail(TNC_E_BUSY, "the plan's network has a batcher, whose batches rewrite its leaves: submit rows");
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
      bool fuse = false;
      double per_launch = 0;
      {
        std::lock_guard<std::mutex> g(s->mu);
        fuse = s->fuse_max > 1 && !(s->heavy_flops > 0 && r->flops >= s->heavy_flops);
        per_launch = s->fuse_flops_per_launch;
      }
      if (fuse) {  // light request: may share grouped launches with others of its structure
        r->tables = lockstep_info(p, first_slice, n_slices);
        if (r->flops < static_cast<double>(r->tables.launches) * per_launch)
          r->key = structure_key(p, first_slice, n_slices);
      }
    }
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->queue.size() >= s->queue_cap) fail(TNC_E_BUSY, "serving queue full");
      r->heavy = s->heavy_flops > 0 && r->flops >= s->heavy_flops;
      if (r->heavy) r->key.clear();
      r->id = s->next_id++;
      r->t_submit = Clock::now();
      s->queue.push_back(r);
      s->reqs[r->id] = r;
    }
    s->cv_work.notify_all();
    *id = r->id;
  TNC_CATCH
}

tnc_status tnc_batcher_create(tnc_plan plan, int32_t batch_label, int32_t n_leaves, const int32_t* leaves,
                              tnc_batcher* out) {
  TNC_TRY
    if (!plan || !out || n_leaves < 1 || !leaves) fail(TNC_E_ARG, "bad batcher arguments");
    Plan& p = *plan->p;
    Net& n = *p.net;
    Ctx& c = *n.ctx;
    const int L = static_cast<int>(n.extents.size());
    if (batch_label < 0 || batch_label >= L) fail(TNC_E_ARG, "batch label out of range");
    if (n.kind[batch_label] != LabelKind::Open && n.kind[batch_label] != LabelKind::Batch)
      fail(TNC_E_ARG, "batch label " + std::to_string(batch_label) + " is not open");
    if (n.open.empty() || n.open[0] != batch_label) fail(TNC_E_ARG, "the batch label must lead the open list");
    std::vector<char> listed(n.n_tensors, 0);
    for (int i = 0; i < n_leaves; ++i) {
      const int t = leaves[i];
      if (t < 0 || t >= n.n_tensors) fail(TNC_E_ARG, "leaf out of range");
      if (listed[t]) fail(TNC_E_ARG, "leaf " + std::to_string(t) + " listed twice");
      listed[t] = 1;
      if (n.labels[t].empty() || n.labels[t][0] != batch_label)
        fail(TNC_E_ARG, "the batch label is not the outermost mode of leaf " + std::to_string(t));
    }
    for (int t = 0; t < n.n_tensors; ++t)
      for (int l : n.labels[t])
        if (l == batch_label && !listed[t])
          fail(TNC_E_ARG, "leaf " + std::to_string(t) + " carries the batch label but is not listed");
    if (n.n_batchers.load() > 0) fail(TNC_E_BUSY, "the network already has a batcher");
    if (c.server) fail(TNC_E_BUSY, "the context is serving: create batchers before tnc_serve_start");
    // re-plan with the listed leaves out of the leaf cache
    if (!c.host_only) {
      set_device(c);
      check_hip(hipStreamSynchronize(c.stream), "sync before re-planning");
      drain_profile(p);
    }
    p.drop_graphs();
    p.volatile_leaf.assign(n.n_tensors, 0);
    for (int i = 0; i < n_leaves; ++i) p.volatile_leaf[leaves[i]] = 1;
    choose_chunking(p, c.arena_bytes);
    // on failure below, the plan goes back to caching every leaf it may
    struct Restore {
      Plan& p;
      size_t arena;
      bool armed = true;
      ~Restore() {
        if (!armed) return;
        p.volatile_leaf.clear();
        try {
          choose_chunking(p, arena);
        } catch (...) {
        }
      }
    } restore{p, c.arena_bytes};
    auto b = std::make_shared<Batcher>();
    b->plan_ref = plan->p;
    b->label = batch_label;
    b->B = n.extents[batch_label];
    for (int i = 0; i < n_leaves; ++i) {
      b->leaves.push_back(leaves[i]);
      b->row_elems.push_back(n.numel[leaves[i]] / b->B);
      b->row_total += b->row_elems.back();
    }
    const int64_t R = p.chunks[0]->R;
    b->out_row = R / b->B;
    b->work_bytes = run_workspace_bytes(p, 0, p.n_slices);
    b->need = b->work_bytes + align_up(R * 16);
    for (const auto& ch : decompose(p, 0, p.n_slices)) b->flops += p.chunk(ch.first).flops;
    if (!c.host_only && b->need > static_cast<int64_t>(c.arena_bytes))
      fail(TNC_E_NOMEM, "a batch needs " + std::to_string(b->need) + " arena bytes, the arena has " +
                            std::to_string(c.arena_bytes));
    *out = new tnc_batcher_s{b};
    restore.armed = false;
    b->plan = &p;  // from here on the batcher holds the network
    ++n.n_batchers;
  TNC_CATCH
}

tnc_status tnc_batcher_destroy(tnc_batcher b) {
  TNC_TRY
  delete b;  // queued rows keep the batcher alive until they are done
  TNC_CATCH
}

tnc_status tnc_submit_row(tnc_ctx ctx, tnc_batcher bh, const void* const* row_data, int32_t in, double* out_c128,
                          tnc_req* id) {
  TNC_TRY
    if (!ctx || !bh || !row_data || !out_c128 || !id) fail(TNC_E_ARG, "NULL argument");
    if (in != TNC_IN_C64 && in != TNC_IN_C128) fail(TNC_E_ARG, "unknown input type");
    Ctx& c = *ctx->c;
    Server* s = c.server.get();
    if (!s) fail(TNC_E_ARG, "server not started");
    const std::shared_ptr<Batcher>& b = bh->b;
    if (b->plan->net->ctx != &c) fail(TNC_E_ARG, "batcher belongs to another context");
    if (b->need > static_cast<int64_t>(c.arena_bytes))
      fail(TNC_E_NOMEM, "a batch needs " + std::to_string(b->need) + " arena bytes, the arena has " +
                            std::to_string(c.arena_bytes));
    auto r = std::make_shared<Request>();
    r->plan_ref = b->plan_ref;
    r->plan = b->plan;
    r->batcher = b;
    r->first = 0;
    r->count = b->plan->n_slices;
    r->out = out_c128;
    r->work_bytes = b->work_bytes;
    r->acc_off = b->work_bytes;
    r->need = b->need;
    r->flops = b->flops;
    r->row.resize(static_cast<size_t>(b->row_total));
    int64_t off = 0;
    for (size_t i = 0; i < b->leaves.size(); ++i) {
      if (!row_data[i]) fail(TNC_E_ARG, "row data of listed leaf " + std::to_string(i) + " is NULL");
      const int64_t re = b->row_elems[i];
      if (in == TNC_IN_C64) {
        std::memcpy(r->row.data() + off, row_data[i], static_cast<size_t>(re) * sizeof(float2));
      } else {
        const double* d = static_cast<const double*>(row_data[i]);
        for (int64_t e = 0; e < re; ++e)
          r->row[off + e] = make_float2(static_cast<float>(d[2 * e]), static_cast<float>(d[2 * e + 1]));
      }
      off += re;
    }
    bool wake = false;
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (b->rows.size() >= s->queue_cap) fail(TNC_E_BUSY, "batcher queue full");
      r->id = s->next_id++;
      r->t_submit = Clock::now();
      b->rows.push_back(r);
      s->reqs[r->id] = r;
      // a running or already queued batch picks the row up; else queue a token
      if (!b->busy && !b->queued) {
        s->enqueue_token(b);
        wake = true;
      }
    }
    if (wake) s->cv_work.notify_all();
    *id = r->id;
  TNC_CATCH
}

static tnc_status finish(Request& r, double* latency_s) {
  if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
  if (r.status != TNC_OK) g_error_set(r.err);
  return r.status;
}

tnc_status tnc_poll(tnc_ctx ctx, tnc_req id, int32_t* done, double* latency_s) {
  TNC_TRY
  if (!ctx || !done || !ctx->c->server) fail(TNC_E_ARG, "bad arguments or server not started");
  Server& s = *ctx->c->server;
  std::lock_guard<std::mutex> g(s.mu);
  auto it = s.reqs.find(id);
  if (it == s.reqs.end()) fail(TNC_E_ARG, "unknown request id");
  *done = it->second->done ? 1 : 0;
  if (!it->second->done) {
    if (latency_s) *latency_s = 0;
    return TNC_OK;
  }
  return finish(*it->second, latency_s);
  TNC_CATCH
}

tnc_status tnc_wait(tnc_ctx ctx, tnc_req id, double* latency_s) {
  TNC_TRY
  if (!ctx || !ctx->c->server) fail(TNC_E_ARG, "bad arguments or server not started");
  Server& s = *ctx->c->server;
  std::unique_lock<std::mutex> g(s.mu);
  auto it = s.reqs.find(id);
  if (it == s.reqs.end()) fail(TNC_E_ARG, "unknown request id");
  std::shared_ptr<Request> r = it->second;
  s.cv_done.wait(g, [&] { return r->done; });
  s.reqs.erase(id);
  return finish(*r, latency_s);
  TNC_CATCH
}

}  // extern "C"
