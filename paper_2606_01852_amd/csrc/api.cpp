// C ABI of the path executor.  Every entry point converts internal errors
// into a status code and a thread-local message; nothing throws across it.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>

#include "core.hpp"
#include "serve.hpp"

namespace tnc {

void fail(tnc_status code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(TNC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

std::recursive_mutex& runtime_mu() {
  static std::recursive_mutex mu;
  return mu;
}

void* pinned_alloc(size_t bytes, const char* what) {
  std::lock_guard<std::recursive_mutex> g(runtime_mu());
  void* p = nullptr;
  check_hip(hipHostMalloc(&p, bytes, hipHostMallocDefault), what);
  return p;
}

void pinned_free(void* p) {
  if (!p) return;
  std::lock_guard<std::recursive_mutex> g(runtime_mu());
  (void)hipHostFree(p);
}

void refuse_while_serving(const Ctx& c, const char* what) {
  if (c.server) fail(TNC_E_BUSY, std::string("the context is serving: ") + what + " is refused until tnc_serve_stop");
}

DeviceBuf::~DeviceBuf() { reset(); }

void DeviceBuf::alloc(size_t n) {
  reset();
  if (n == 0) return;
  void* p = nullptr;
  std::lock_guard<std::recursive_mutex> g(runtime_mu());
  const hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? TNC_E_NOMEM : TNC_E_DEVICE,
         "hipMalloc of " + std::to_string(n) + " bytes: " + hipGetErrorString(e));
  }
  ptr = p;
  bytes = n;
}

void DeviceBuf::reset() {
  if (ptr) {
    std::lock_guard<std::recursive_mutex> g(runtime_mu());
    (void)hipFree(ptr);
  }
  ptr = nullptr;
  bytes = 0;
}

Net::~Net() {
  if (ctx && !ctx->host_only) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  }
}

Ctx::~Ctx() {
  server.reset();
  if (!host_only) {
    (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    scratch.reset();
    std::lock_guard<std::recursive_mutex> g(runtime_mu());
    if (own_arena && arena) (void)hipFree(arena);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
}

void set_device(const Ctx& c) {
  if (c.host_only) fail(TNC_E_UNSUPPORTED, "host-only context cannot run device work");
  check_hip(hipSetDevice(c.device), "hipSetDevice");
}

}  // namespace tnc

using namespace tnc;


namespace tnc {
namespace {
thread_local std::string g_msg;
}
void g_error_clear() { g_msg.clear(); }
void g_error_set(const std::string& m) { g_msg = m; }
const char* g_error_get() { return g_msg.c_str(); }
}  // namespace tnc

extern "C" {

const char* tnc_last_error(void) { return tnc::g_error_get(); }

const char* tnc_version(void) { return "tnc 0.1 (gfx950)"; }

int tnc_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

tnc_status tnc_ctx_create(int device, void* arena, size_t arena_bytes, void* stream, tnc_ctx* out) {
  TNC_TRY
  if (!out) fail(TNC_E_ARG, "out is NULL");
  auto h = std::make_unique<tnc_ctx_s>();
  h->c = std::make_shared<Ctx>();
  Ctx& c = *h->c;
  c.device = device;
  c.host_only = device < 0;
  c.arena_bytes = arena_bytes;
  if (!c.host_only) {
    const int nd = tnc_device_count();
    if (device >= nd) fail(TNC_E_DEVICE, "device " + std::to_string(device) + " not present");
    check_hip(hipSetDevice(device), "hipSetDevice");
    if (arena) {
      c.arena = static_cast<char*>(arena);
    } else if (arena_bytes) {
      void* p = nullptr;
      std::lock_guard<std::recursive_mutex> g(runtime_mu());
      const hipError_t e = hipMalloc(&p, arena_bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(TNC_E_NOMEM, "arena hipMalloc failed: " + std::string(hipGetErrorString(e)));
      }
      c.arena = static_cast<char*>(p);
      c.own_arena = true;
    }
    // per-device address of the allocation-free permute tables, looked up
    // once here with the device current; if the lookup fails, the error is
    // cleared and tnc_permute_noalloc looks again and reports it
    void* tables = nullptr;
    if (static_table_area(device, &tables) != hipSuccess) (void)hipGetLastError();
    load_tune_cache(c);
    prepare_gemm_kernels();
    (void)hipGetLastError();  // best effort: launches retry lazily
    if (stream) {
      c.stream = static_cast<hipStream_t>(stream);
    } else {
      std::lock_guard<std::recursive_mutex> g(runtime_mu());
      check_hip(hipStreamCreate(&c.stream), "hipStreamCreate");
      c.own_stream = true;
    }
  } else if (arena) {
    fail(TNC_E_ARG, "a host-only context takes no arena");
  }
  *out = h.release();
  TNC_CATCH
}

tnc_status tnc_ctx_destroy(tnc_ctx ctx) {
  TNC_TRY
  // stop serving first: queued requests hold plans, which hold this context
  if (ctx && ctx->c) ctx->c->server.reset();
  delete ctx;
  TNC_CATCH
}

tnc_status tnc_ctx_set_gemm_variant(tnc_ctx ctx, int32_t variant) {
  TNC_TRY
  if (!ctx) fail(TNC_E_ARG, "ctx is NULL");
  if (variant < -1 || variant >= kGemmVariants) fail(TNC_E_ARG, "variant out of range");
  refuse_while_serving(*ctx->c, "changing the forced tile variant");
  ctx->c->gemm_variant = variant;
  TNC_CATCH
}

int tnc_gemm_variant_count(void) { return kGemmVariants; }

tnc_status tnc_ctx_sync(tnc_ctx ctx) {
  TNC_TRY
  if (!ctx) fail(TNC_E_ARG, "ctx is NULL");
  set_device(*ctx->c);
  check_hip(hipStreamSynchronize(ctx->c->stream), "stream synchronize");
  TNC_CATCH
}

static void upload_leaf(Net& net, int t, const void* host, int32_t in) {
  DeviceBuf& d = net.leaf[t];
  const int64_t n = net.numel[t];
  ++net.version[t];
  if (!d.ptr) d.alloc(static_cast<size_t>(n) * 8);
  if (in == TNC_IN_C64) {
    check_hip(hipMemcpy(d.ptr, host, n * 8, hipMemcpyHostToDevice), "leaf upload");
  } else if (in == TNC_IN_C128) {
    const double* src = static_cast<const double*>(host);
    std::vector<float> tmp(static_cast<size_t>(2 * n));
    for (int64_t i = 0; i < 2 * n; ++i) tmp[i] = static_cast<float>(src[i]);
    check_hip(hipMemcpy(d.ptr, tmp.data(), n * 8, hipMemcpyHostToDevice), "leaf upload");
  } else {
    fail(TNC_E_ARG, "unknown input element type");
  }
}

tnc_status tnc_net_create(tnc_ctx ctx, int32_t n_tensors, const int32_t* ranks, const int32_t* labels,
                          int32_t n_labels, const int64_t* extent_of_label, int32_t n_open,
                          const int32_t* open_labels, const void* const* host_data, int32_t in, tnc_net* out) {
  TNC_TRY
  if (!ctx || !out) fail(TNC_E_ARG, "ctx/out is NULL");
  if (in != TNC_IN_C64 && in != TNC_IN_C128) fail(TNC_E_ARG, "unknown input element type");
  if (n_tensors < 1 || !ranks || n_labels < 0 || (n_labels && !extent_of_label) || n_open < 0 ||
      (n_open && !open_labels))
    fail(TNC_E_ARG, "bad network arguments");
  auto h = std::make_unique<tnc_net_s>();
  h->n = std::make_shared<Net>();
  Net& net = *h->n;
  net.ctx_ref = ctx->c;
  net.ctx = ctx->c.get();
  net.n_tensors = n_tensors;
  net.labels.resize(n_tensors);
  int64_t pos = 0;
  for (int t = 0; t < n_tensors; ++t) {
    if (ranks[t] < 0) fail(TNC_E_ARG, "negative rank");
    if (ranks[t] && !labels) fail(TNC_E_ARG, "labels is NULL");
    net.labels[t].assign(labels + pos, labels + pos + ranks[t]);
    pos += ranks[t];
  }
  net.extents.assign(extent_of_label, extent_of_label + n_labels);
  net.open.assign(open_labels, open_labels + n_open);
  validate_net(net);
  net.leaf.resize(n_tensors);
  net.version.assign(n_tensors, 0);
  if (!ctx->c->host_only) {
    if (!host_data) fail(TNC_E_ARG, "host_data is NULL");
    set_device(*ctx->c);
    for (int t = 0; t < n_tensors; ++t) {
      if (!host_data[t]) fail(TNC_E_ARG, "host_data[" + std::to_string(t) + "] is NULL");
      upload_leaf(net, t, host_data[t], in);
    }
  }
  *out = h.release();
  TNC_CATCH
}

tnc_status tnc_net_set_tensor(tnc_net net, int32_t tensor, const void* host_data, int32_t in) {
  TNC_TRY
  if (!net || !host_data) fail(TNC_E_ARG, "net/host_data is NULL");
  if (in != TNC_IN_C64 && in != TNC_IN_C128) fail(TNC_E_ARG, "unknown input element type");
  Net& n = *net->n;
  if (tensor < 0 || tensor >= n.n_tensors) fail(TNC_E_ARG, "tensor out of range");
  refuse_while_serving(*n.ctx, "replacing a leaf");
  set_device(*n.ctx);
  check_hip(hipStreamSynchronize(n.ctx->stream), "stream synchronize");
  upload_leaf(n, tensor, host_data, in);
  TNC_CATCH
}

tnc_status tnc_net_set_tensor_device(tnc_net net, int32_t tensor, const void* dev_data) {
  TNC_TRY
  if (!net || !dev_data) fail(TNC_E_ARG, "net/dev_data is NULL");
  Net& n = *net->n;
  if (tensor < 0 || tensor >= n.n_tensors) fail(TNC_E_ARG, "tensor out of range");
  refuse_while_serving(*n.ctx, "replacing a leaf");
  set_device(*n.ctx);
  check_hip(hipMemcpyAsync(n.leaf[tensor].ptr, dev_data, n.numel[tensor] * 8, hipMemcpyDeviceToDevice, n.ctx->stream),
            "leaf copy");
  ++n.version[tensor];
  TNC_CATCH
}

tnc_status tnc_net_destroy(tnc_net net) {
  TNC_TRY
  delete net;  // the network itself goes when its last plan does
  TNC_CATCH
}

tnc_status tnc_plan_create(tnc_net net, int32_t n_steps, const int32_t* ssa_pairs, int32_t n_sliced,
                           const int32_t* sliced_labels, int32_t prec, int32_t cgemm, tnc_plan* out) {
  TNC_TRY
  if (!net || !out) fail(TNC_E_ARG, "net/out is NULL");
  if (n_steps < 0 || (n_steps && !ssa_pairs) || n_sliced < 0 || (n_sliced && !sliced_labels))
    fail(TNC_E_ARG, "bad plan arguments");
  if (prec != TNC_PREC_C64 && prec != TNC_PREC_BF16X3) fail(TNC_E_ARG, "unknown precision");
  if (cgemm != TNC_GEMM_4M && cgemm != TNC_GEMM_3M) fail(TNC_E_ARG, "unknown GEMM form");
  Net& n = *net->n;
  auto h = std::make_unique<tnc_plan_s>();
  h->p = std::make_shared<Plan>();
  Plan& p = *h->p;
  p.net_ref = net->n;
  p.net = &n;
  p.prec = static_cast<tnc_prec>(prec);
  p.form = static_cast<tnc_cgemm>(cgemm);
  for (int s = 0; s < n_steps; ++s) p.pairs.push_back({ssa_pairs[2 * s], ssa_pairs[2 * s + 1]});
  validate_path(n, p.pairs);
  std::vector<char> seen(n.extents.size(), 0);
  for (int i = 0; i < n_sliced; ++i) {
    const int l = sliced_labels[i];
    if (l < 0 || l >= static_cast<int>(n.extents.size())) fail(TNC_E_ARG, "sliced label out of range");
    if (n.kind[l] != LabelKind::Closed) fail(TNC_E_ARG, "sliced label " + std::to_string(l) + " is not closed");
    if (seen[l]) fail(TNC_E_ARG, "sliced label repeated");
    seen[l] = 1;
    p.sliced.push_back(l);
  }
  p.suffix_prod.assign(n_sliced + 1, 1);
  for (int j = 1; j <= n_sliced; ++j) {
    p.suffix_prod[j] = p.suffix_prod[j - 1] * n.extents[p.sliced[n_sliced - j]];
    if (p.suffix_prod[j] > (int64_t{1} << 40)) fail(TNC_E_ARG, "too many slices");
  }
  p.n_slices = p.suffix_prod[n_sliced];
  choose_chunking(p, n.ctx->arena_bytes);
  const ChunkPlan& c0 = *p.chunks[0];
  if (n.ctx->arena_bytes && static_cast<size_t>(c0.peak) + run_extra_bytes(c0, 1) > n.ctx->arena_bytes)
    fail(TNC_E_NOMEM, "planned peak of one slice (" + std::to_string(c0.peak) + " B) exceeds the arena (" +
                          std::to_string(n.ctx->arena_bytes) + " B)");
  if (!n.ctx->host_only) {
    set_device(*n.ctx);
    p.acc.alloc(static_cast<size_t>(std::max<int64_t>(1, c0.R)) * 16);
    p.norm.alloc(256);
  }
  *out = h.release();
  TNC_CATCH
}

tnc_status tnc_plan_destroy(tnc_plan plan) {
  TNC_TRY
  delete plan;  // in-flight served requests keep the plan until they finish
  TNC_CATCH
}

tnc_status tnc_plan_get_info(tnc_plan plan, tnc_plan_info* out) {
  TNC_TRY
  if (!plan || !out) fail(TNC_E_ARG, "plan/out is NULL");
  Plan& p = *plan->p;
  const ChunkPlan& c0 = *p.chunks[0];
  const ChunkPlan& cm = p.chunk(p.j_max);
  tnc_plan_info info{};
  info.flops_per_slice = c0.flops;
  info.bytes_per_slice = c0.bytes;
  info.transpose_bytes = c0.transpose_bytes;
  info.n_slices = p.n_slices;
  info.max_intermediate = c0.max_tensor;
  info.peak_bytes = c0.peak;
  info.max_chunk = p.suffix_prod[p.j_max];
  info.chunk_peak_bytes = cm.peak;
  info.chunk_flops = cm.flops;
  info.n_steps = static_cast<int32_t>(p.pairs.size());
  info.n_permutes = c0.n_permutes;
  info.n_permuted_stores = c0.n_perm_stores;
  info.n_cached_leaves = c0.n_cached;
  for (const LeafPrep& lp : c0.leaf) info.n_inplace_leaves += lp.inplace ? 1 : 0;
  info.n_launches = lockstep_info(p, 0, p.n_slices).launches;
  info.n_result = static_cast<int32_t>(std::min<int64_t>(c0.R, INT32_MAX));
  *out = info;
  TNC_CATCH
}

static void step_info(const ChunkPlan& c, int32_t step, tnc_step_info* out) {
  if (step < 0 || step >= static_cast<int32_t>(c.steps.size())) fail(TNC_E_ARG, "step out of range");
  const StepPlan& s = c.steps[step];
  tnc_step_info i{};
  i.A = s.A;
  i.B = s.B;
  i.C = s.C;
  i.nH = static_cast<int32_t>(s.H.size());
  i.nM = static_cast<int32_t>(s.M.size());
  i.nN = static_cast<int32_t>(s.N.size());
  i.nK = static_cast<int32_t>(s.K.size());
  i.h = s.h;
  i.m = s.m;
  i.n = s.n;
  i.k = s.k;
  i.natural = s.natural ? 1 : 0;
  i.kernel = static_cast<int32_t>(s.kind);
  i.variant = s.variant;
  i.swapped = s.swap ? 1 : 0;
  i.split = s.split;
  i.hA = s.hA;
  i.hB = s.hB;
  i.presplit = s.presplit ? 1 : 0;
  for (int side = 1; side <= 2; ++side) {
    const int id = side == 1 ? s.la : s.lb;
    if (id >= 0 && id < static_cast<int>(c.leaf.size()) && c.leaf[id].planes_side == side)
      i.presplit_fused |= side;
  }
  *out = i;
}

tnc_status tnc_plan_get_step(tnc_plan plan, int32_t step, tnc_step_info* out) {
  TNC_TRY
  if (!plan || !out) fail(TNC_E_ARG, "plan/out is NULL");
  step_info(*plan->p->chunks[0], step, out);
  TNC_CATCH
}

tnc_status tnc_plan_get_batch_step(tnc_plan plan, int32_t step, tnc_step_info* out) {
  TNC_TRY
  if (!plan || !out) fail(TNC_E_ARG, "plan/out is NULL");
  Plan& p = *plan->p;
  step_info(p.chunk(p.j_max), step, out);
  TNC_CATCH
}

tnc_status tnc_plan_get_order(tnc_plan plan, int32_t id, int32_t* labels, int32_t cap, int32_t* rank) {
  TNC_TRY
  if (!plan || !rank || (cap > 0 && !labels)) fail(TNC_E_ARG, "bad arguments");
  const ChunkPlan& c0 = *plan->p->chunks[0];
  if (id < 0 || id >= static_cast<int32_t>(c0.order.size())) fail(TNC_E_ARG, "tensor id out of range");
  const auto& o = c0.order[id];
  for (int q = 0; q < std::min<int>(cap, static_cast<int>(o.size())); ++q) labels[q] = o[q];
  *rank = static_cast<int32_t>(o.size());
  TNC_CATCH
}

tnc_status tnc_plan_set_max_chunk(tnc_plan plan, int64_t max_chunk) {
  TNC_TRY
  if (!plan) fail(TNC_E_ARG, "plan is NULL");
  Plan& p = *plan->p;
  refuse_while_serving(*p.net->ctx, "changing the chunk cap");
  p.max_chunk_user = max_chunk;
  int j = 0;
  for (int q = 1; q < static_cast<int>(p.suffix_prod.size()); ++q) {
    if (max_chunk > 0 && p.suffix_prod[q] > max_chunk) break;
    if (!p.chunks[q]) {
      auto cp = build_chunk(p, q);
      const size_t need = static_cast<size_t>(cp->peak) + run_extra_bytes(*cp, 1);
      if (p.net->ctx->arena_bytes && need > p.net->ctx->arena_bytes) break;
      p.chunks[q] = std::move(cp);
    } else {
      const size_t need = static_cast<size_t>(p.chunks[q]->peak) + run_extra_bytes(*p.chunks[q], 1);
      if (p.net->ctx->arena_bytes && need > p.net->ctx->arena_bytes) break;
    }
    j = q;
  }
  p.j_max = j;
  TNC_CATCH
}

tnc_status tnc_plan_distribute(tnc_plan plan, int32_t n_gpus, double large_bytes, const tnc_dist_hw* hw,
                               tnc_dist_step* steps, int32_t cap, int32_t* n_steps, double* total_s,
                               double* redistributed_bytes) {
  TNC_TRY
  if (!plan || !hw || !n_steps || !total_s || !redistributed_bytes || cap < 0 || (cap && !steps))
    fail(TNC_E_ARG, "bad arguments");
  if (n_gpus < 2) fail(TNC_E_ARG, "distribution needs at least two GPUs");
  if (!(hw->hbm_bytes_per_s > 0) || !(hw->flops_per_s > 0) || !(hw->net_bytes_per_s > 0) || hw->latency_s < 0)
    fail(TNC_E_ARG, "hardware constants must be positive");
  std::vector<tnc_dist_step> out;
  double total = 0, moved = 0;
  plan_distribution(*plan->p, n_gpus, large_bytes, *hw, out, total, moved);
  for (int i = 0; i < std::min<int>(cap, static_cast<int>(out.size())); ++i) steps[i] = out[i];
  *n_steps = static_cast<int32_t>(out.size());
  *total_s = total;
  *redistributed_bytes = moved;
  TNC_CATCH
}

tnc_status tnc_plan_autotune(tnc_plan plan) {
  TNC_TRY
  if (!plan) fail(TNC_E_ARG, "plan is NULL");
  Plan& p = *plan->p;
  refuse_while_serving(*p.net->ctx, "autotuning");
  set_device(*p.net->ctx);
  {
    std::lock_guard<std::mutex> g(p.mu);
    for (auto& cp : p.chunks)
      if (cp) assign_variants(p, *cp, true);
  }
  p.drop_graphs();  // captured graphs hold the previous tile variants
  TNC_CATCH
}

tnc_status tnc_plan_set_graph(tnc_plan plan, int32_t enable) {
  TNC_TRY
  if (!plan) fail(TNC_E_ARG, "plan is NULL");
  refuse_while_serving(*plan->p->net->ctx, "switching graph replay");
  plan->p->graph = enable ? 1 : 0;
  TNC_CATCH
}

tnc_status tnc_plan_set_grouping(tnc_plan plan, int32_t enable) {
  TNC_TRY
  if (!plan) fail(TNC_E_ARG, "plan is NULL");
  Plan& p = *plan->p;
  Ctx& c = *p.net->ctx;
  refuse_while_serving(c, "changing the execution order");
  const int g = enable ? 1 : 0;
  if (g == p.grouping) return TNC_OK;
  if (!c.host_only) {
    set_device(c);
    check_hip(hipStreamSynchronize(c.stream), "sync before re-planning");
    drain_profile(p);
  }
  p.drop_graphs();
  p.grouping = g;
  choose_chunking(p, c.arena_bytes);
  TNC_CATCH
}

tnc_status tnc_plan_set_store_order(tnc_plan plan, int32_t mode) {
  TNC_TRY
  if (!plan) fail(TNC_E_ARG, "plan is NULL");
  if (mode != 0 && mode != 1) fail(TNC_E_ARG, "store order must be 0 or 1");
  Plan& p = *plan->p;
  Ctx& c = *p.net->ctx;
  refuse_while_serving(c, "changing the store order");
  if (mode == p.store_order) return TNC_OK;
  if (!c.host_only) {
    set_device(c);
    check_hip(hipStreamSynchronize(c.stream), "sync before re-planning");
    drain_profile(p);
  }
  p.drop_graphs();
  p.store_order = mode;
  choose_chunking(p, c.arena_bytes);
  TNC_CATCH
}

tnc_status tnc_plan_set_profile(tnc_plan plan, int32_t enable) {
  TNC_TRY
  if (!plan) fail(TNC_E_ARG, "plan is NULL");
  Plan& p = *plan->p;
  refuse_while_serving(*p.net->ctx, "switching profiling");
  if (!p.net->ctx->host_only) drain_profile(p);
  p.profile = enable ? 1 : 0;
  p.timers.assign(p.pairs.size() + 3, StepTimer{});
  TNC_CATCH
}

tnc_status tnc_plan_get_profile(tnc_plan plan, int32_t step, double* ms, int64_t* launches) {
  TNC_TRY
  if (!plan || !ms || !launches) fail(TNC_E_ARG, "bad arguments");
  Plan& p = *plan->p;
  set_device(*p.net->ctx);
  drain_profile(p);
  const int ns = static_cast<int>(p.pairs.size());
  int idx = step;
  if (step == -1) idx = ns;
  if (step == -2) idx = ns + 1;
  if (step == -3) idx = ns + 2;
  if (idx < 0 || idx >= ns + 3) fail(TNC_E_ARG, "step out of range");
  if (p.timers.size() < static_cast<size_t>(ns + 3)) p.timers.resize(ns + 3);
  *ms = p.timers[idx].ms;
  *launches = p.timers[idx].launches;
  TNC_CATCH
}

static void check_range(const Plan& p, int64_t first, int64_t count) {
  if (first < 0 || count < 1 || first + count > p.n_slices)
    fail(TNC_E_ARG, "slice range [" + std::to_string(first) + ", " + std::to_string(first + count) +
                        ") outside [0, " + std::to_string(p.n_slices) + ")");
}

tnc_status tnc_contract(tnc_plan plan, int64_t first_slice, int64_t n_slices, double* out_c128) {
  TNC_TRY
  if (!plan || !out_c128) fail(TNC_E_ARG, "plan/out is NULL");
  Plan& p = *plan->p;
  Ctx& c = *p.net->ctx;
  refuse_while_serving(c, "a direct contraction (submit a request instead)");
  set_device(c);
  check_range(p, first_slice, n_slices);
  const ChunkPlan& c0 = *p.chunks[0];
  RunArgs a;
  a.first = first_slice;
  a.count = n_slices;
  a.arena = c.arena;
  a.arena_bytes = c.arena_bytes;
  a.acc = static_cast<double2*>(p.acc.ptr);
  a.stream = c.stream;
  a.fresh_acc = true;
  run_plan(p, a);
  // the result comes back through the plan's pinned staging buffer
  const size_t res_bytes = static_cast<size_t>(c0.R) * 16;
  if (p.host_res_bytes < res_bytes) {
    pinned_free(p.host_res);
    p.host_res = nullptr;
    p.host_res_bytes = 0;
    p.host_res = pinned_alloc(res_bytes, "pinned result buffer");
    p.host_res_bytes = res_bytes;
  }
  check_hip(hipMemcpyAsync(p.host_res, a.acc, res_bytes, hipMemcpyDeviceToHost, c.stream), "result copy");
  check_hip(hipStreamSynchronize(c.stream), "stream synchronize");
  const double* tmp = static_cast<const double*>(p.host_res);
  if (c0.result_perm.empty()) {
    std::memcpy(out_c128, tmp, res_bytes);
  } else {
    for (int64_t u = 0; u < c0.R; ++u) {
      out_c128[2 * u] = tmp[2 * c0.result_perm[u]];
      out_c128[2 * u + 1] = tmp[2 * c0.result_perm[u] + 1];
    }
  }
  TNC_CATCH
}

tnc_status tnc_contract_async(tnc_plan plan, int64_t first_slice, int64_t n_slices, void* out_dev,
                              int32_t out_type) {
  TNC_TRY
  if (!plan || !out_dev) fail(TNC_E_ARG, "plan/out is NULL");
  if (out_type != TNC_OUT_C64 && out_type != TNC_OUT_C128) fail(TNC_E_ARG, "unknown output type");
  Plan& p = *plan->p;
  Ctx& c = *p.net->ctx;
  refuse_while_serving(c, "a direct contraction (submit a request instead)");
  set_device(c);
  check_range(p, first_slice, n_slices);
  const ChunkPlan& c0 = *p.chunks[0];
  if (!c0.result_perm.empty()) fail(TNC_E_UNSUPPORTED, "device results need batch labels leading the open order");
  RunArgs a;
  a.first = first_slice;
  a.count = n_slices;
  a.arena = c.arena;
  a.arena_bytes = c.arena_bytes;
  a.stream = c.stream;
  if (out_type == TNC_OUT_C64 && n_slices == 1 && !p.pairs.empty()) {
    a.direct_out = static_cast<float2*>(out_dev);
    run_plan(p, a);
  } else if (out_type == TNC_OUT_C64) {
    a.acc = static_cast<double2*>(p.acc.ptr);
    a.fresh_acc = true;
    run_plan(p, a);
    check_hip(launch_c128_to_c64(a.acc, static_cast<float2*>(out_dev), c0.R, c.stream), "result conversion");
  } else if (out_type == TNC_OUT_C128) {
    a.acc = static_cast<double2*>(out_dev);
    a.fresh_acc = true;
    run_plan(p, a);
  } else {
    fail(TNC_E_ARG, "unknown output type");
  }
  TNC_CATCH
}

tnc_status tnc_plan_result_norm2(tnc_plan plan, double* out) {
  TNC_TRY
  if (!plan || !out) fail(TNC_E_ARG, "plan/out is NULL");
  Plan& p = *plan->p;
  Ctx& c = *p.net->ctx;
  set_device(c);
  const ChunkPlan& c0 = *p.chunks[0];
  check_hip(launch_norm2(static_cast<double2*>(p.acc.ptr), c0.R, static_cast<double*>(p.norm.ptr), c.stream), "norm");
  double v = 0;
  check_hip(hipMemcpyAsync(&v, p.norm.ptr, sizeof(double), hipMemcpyDeviceToHost, c.stream), "norm copy");
  check_hip(hipStreamSynchronize(c.stream), "stream synchronize");
  *out = v;
  TNC_CATCH
}

}  // extern "C"

namespace {

// A checked permutation of a complex64 tensor: its gather-permute and, when
// tiled, the index tables packed into one host blob (parts 256-byte
// aligned, offsets in off[]).
struct PermuteJob {
  PermuteHost ph;
  std::vector<uint8_t> blob;
  size_t off[6] = {0, 0, 0, 0, 0, 0};
};

PermuteJob plan_permute(int32_t rank, const int64_t* extents, const int32_t* perm) {
  std::vector<int64_t> ist(rank);
  int64_t s = 1;
  for (int q = rank - 1; q >= 0; --q) {
    if (extents[q] < 1) fail(TNC_E_ARG, "extent < 1");
    if (s > INT64_MAX / 8 / extents[q]) fail(TNC_E_ARG, "tensor size overflows int64");
    ist[q] = s;
    s *= extents[q];
  }
  std::vector<char> seen(rank, 0);
  std::vector<int64_t> ext(rank), st(rank);
  for (int q = 0; q < rank; ++q) {
    const int p = perm[q];
    if (p < 0 || p >= rank || seen[p]) fail(TNC_E_ARG, "perm is not a permutation");
    seen[p] = 1;
    ext[q] = extents[p];
    st[q] = ist[p];
  }
  PermuteJob j;
  j.ph = build_permute(ext, st);
  if (j.ph.tiled) {
    auto put = [&](const void* src, size_t bytes) {
      const size_t off = (j.blob.size() + 255) / 256 * 256;
      j.blob.resize(off + bytes);
      std::memcpy(j.blob.data() + off, src, bytes);
      return off;
    };
    const PermuteHost& ph = j.ph;
    j.off[0] = put(ph.tile_in.data(), ph.tile_in.size() * 4);
    j.off[1] = put(ph.tile_slot_r.data(), ph.tile_slot_r.size() * 4);
    j.off[2] = put(ph.tile_out.data(), ph.tile_out.size() * 4);
    j.off[3] = put(ph.tile_slot_w.data(), ph.tile_slot_w.size() * 4);
    j.off[4] = put(ph.lo_tab.data(), ph.lo_tab.size() * 8);
    j.off[5] = put(ph.hi_tab.data(), ph.hi_tab.size() * 8);
  }
  return j;
}

// Launch a planned permutation; `tables` is the device copy of j.blob.
hipError_t launch_permute_job(const PermuteJob& j, const void* in, void* out, const char* tables, hipStream_t s) {
  if (!j.ph.tiled) {
    GatherDesc g = j.ph.plain;
    g.in = static_cast<const float2*>(in);
    g.out = static_cast<float2*>(out);
    return launch_gather(g, s);
  }
  PermuteDesc d{};
  d.in = static_cast<const float2*>(in);
  d.out = static_cast<float2*>(out);
  d.tile_in = reinterpret_cast<const int32_t*>(tables + j.off[0]);
  d.tile_slot_r = reinterpret_cast<const int32_t*>(tables + j.off[1]);
  d.tile_out = reinterpret_cast<const int32_t*>(tables + j.off[2]);
  d.tile_slot_w = reinterpret_cast<const int32_t*>(tables + j.off[3]);
  d.lo_tab = reinterpret_cast<const int64_t*>(tables + j.off[4]);
  d.hi_tab = reinterpret_cast<const int64_t*>(tables + j.off[5]);
  d.n_tiles = j.ph.n_tiles;
  d.L = j.ph.L;
  d.T = j.ph.T;
  d.slots = j.ph.slots;
  d.pairs = j.ph.pairs ? 1 : 0;
  return launch_permute(d, s);
}

}  // namespace

extern "C" {

tnc_status tnc_permute(tnc_ctx ctx, const void* in, void* out, int32_t rank, const int64_t* extents,
                       const int32_t* perm) {
  TNC_TRY
  if (!ctx || !in || !out || rank < 0 || (rank && (!extents || !perm))) fail(TNC_E_ARG, "bad arguments");
  const PermuteJob j = plan_permute(rank, extents, perm);
  Ctx& c = *ctx->c;
  set_device(c);
  if (j.ph.tiled) {
    check_hip(hipStreamSynchronize(c.stream), "stream synchronize");
    if (c.scratch.bytes < j.blob.size()) c.scratch.alloc(j.blob.size());
    check_hip(hipMemcpy(c.scratch.ptr, j.blob.data(), j.blob.size(), hipMemcpyHostToDevice), "table upload");
  }
  check_hip(launch_permute_job(j, in, out, static_cast<const char*>(c.scratch.ptr), c.stream), "permute launch");
  TNC_CATCH
}

tnc_status tnc_permute_noalloc(tnc_ctx ctx, const void* in, void* out, int32_t rank, const int64_t* extents,
                               const int32_t* perm) {
  TNC_TRY
  if (!ctx || !in || !out || rank < 0 || (rank && (!extents || !perm))) fail(TNC_E_ARG, "bad arguments");
  const PermuteJob j = plan_permute(rank, extents, perm);
  if (j.blob.size() > kStaticPermuteTableBytes)
    fail(TNC_E_NOMEM, "the permutation's index tables need " + std::to_string(j.blob.size()) +
                          " bytes, above the fixed table area of " + std::to_string(kStaticPermuteTableBytes));
  Ctx& c = *ctx->c;
  set_device(c);
  void* tables = nullptr;
  if (j.ph.tiled) {
    check_hip(static_table_area(c.device, &tables), "table area address");
    // earlier launches on this stream may still read the shared tables: wait
    // for them, copy the new tables, and wait for the copy (the host blob
    // is pageable and goes away when this call returns)
    check_hip(hipStreamSynchronize(c.stream), "stream synchronize");
    check_hip(hipMemcpyAsync(tables, j.blob.data(), j.blob.size(), hipMemcpyHostToDevice, c.stream), "table upload");
    check_hip(hipStreamSynchronize(c.stream), "table upload");
  }
  check_hip(launch_permute_job(j, in, out, static_cast<const char*>(tables), c.stream), "permute launch");
  TNC_CATCH
}

tnc_status tnc_device_calibrate(tnc_ctx ctx, tnc_dist_hw* hw) {
  TNC_TRY
  if (!ctx || !hw) fail(TNC_E_ARG, "ctx/hw is NULL");
  Ctx& c = *ctx->c;
  if (c.host_only) fail(TNC_E_ARG, "host-only context");
  set_device(c);
  check_hip(hipStreamSynchronize(c.stream), "stream synchronize");
  int cus = 0;
  check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device), "device attribute");
  const int blocks = 8 * std::max(cus, 1);
  const int iters = 4000;
  const int64_t copy_bytes = int64_t{2} << 30;  // far above the 256 MiB last-level cache
  DeviceBuf sink, src, dst;
  sink.alloc(static_cast<size_t>(blocks) * 256 * sizeof(float));
  src.alloc(static_cast<size_t>(copy_bytes));
  dst.alloc(static_cast<size_t>(copy_bytes));
  check_hip(hipMemsetAsync(src.ptr, 0, static_cast<size_t>(copy_bytes), c.stream), "memset");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  check_hip(hipEventCreate(&e0), "event");
  check_hip(hipEventCreate(&e1), "event");
  auto best_ms = [&](auto&& launch) {
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      check_hip(launch(), "calibration launch");  // warm-up
      check_hip(hipEventRecord(e0, c.stream), "event");
      check_hip(launch(), "calibration launch");
      check_hip(hipEventRecord(e1, c.stream), "event");
      check_hip(hipEventSynchronize(e1), "event");
      float ms = 0.f;
      check_hip(hipEventElapsedTime(&ms, e0, e1), "event");
      best = std::min(best, ms);
    }
    return static_cast<double>(best);
  };
  const double mfma_ms =
      best_ms([&] { return launch_mfma_rate(static_cast<float*>(sink.ptr), blocks, iters, c.stream); });
  const double copy_ms = best_ms([&] { return launch_copy_rate(src.ptr, dst.ptr, copy_bytes, c.stream); });
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // per wave and round: 8 MFMAs of 16 x 16 x 4 multiply-adds
  const double flops = static_cast<double>(blocks) * 4 * iters * 8 * (16.0 * 16 * 4 * 2);
  hw->flops_per_s = flops / (mfma_ms * 1e-3);
  hw->hbm_bytes_per_s = 2.0 * static_cast<double>(copy_bytes) / (copy_ms * 1e-3);
  TNC_CATCH
}

tnc_status tnc_batched_cgemm(tnc_ctx ctx, int64_t h, int64_t m, int64_t n, int64_t k, const void* A,
                             int64_t stride_a, const void* B, int64_t stride_b, void* C, int32_t prec,
                             int32_t form) {
  TNC_TRY
  if (!ctx || !A || !B || !C || h < 1 || m < 1 || n < 1 || k < 1 || stride_a < 0 || stride_b < 0)
    fail(TNC_E_ARG, "bad arguments");
  if (prec != TNC_PREC_C64 && prec != TNC_PREC_BF16X3) fail(TNC_E_ARG, "unknown precision");
  if (form != TNC_GEMM_4M && form != TNC_GEMM_3M) fail(TNC_E_ARG, "unknown GEMM form");
  Ctx& c = *ctx->c;
  set_device(c);
  GemmDesc d;
  std::memset(&d, 0, sizeof(d));
  d.A = static_cast<const float2*>(A);
  d.B = static_cast<const float2*>(B);
  d.C = static_cast<float2*>(C);
  d.m = m;
  d.n = n;
  d.k = k;
  d.h = h;
  d.pow2 = 0;
  if (h > 1) {
    if (h > INT32_MAX) fail(TNC_E_ARG, "batch too large");
    d.nbd = 1;
    d.bext[0] = static_cast<int32_t>(h);
    d.bsA[0] = stride_a;
    d.bsB[0] = stride_b;
    if ((h & (h - 1)) == 0) {
      d.pow2 = 1;
      int sh = 0;
      while ((int64_t{1} << sh) < h) ++sh;
      d.bshift[0] = sh;
    }
  }
  const GemmKernel kind = choose_gemm_kernel(h, m, n, k);
  check_hip(launch_gemm(d, kind, c.gemm_variant < 0 ? 0 : c.gemm_variant, form == TNC_GEMM_3M ? Form::M3 : Form::M4,
                        prec == TNC_PREC_BF16X3 ? Prec::BF16X3 : Prec::C64, c.stream),
            "gemm launch");
  TNC_CATCH
}

}  // extern "C"
