// Path executor: uploads a chunk plan's tables once, then replays the path
// for each chunk of slices -- leaf permutations, one batched complex GEMM
// per step, FP64 accumulation of the root -- on one stream with no
// allocation inside the loop (paper Sec. IV: the executor replays the
// planned schedule; slicing, Sec. II-C, becomes a batch dimension).
#include <algorithm>
#include <cstring>
#include <map>

#include "core.hpp"

namespace tnc {

namespace {

int64_t align_up(int64_t x) { return (x + 255) / 256 * 256; }

// Device address of cached leaf t inside the chunk plan's leaf cache.
float2* cached_leaf(const ChunkPlan& cp, int t) {
  return reinterpret_cast<float2*>(static_cast<char*>(cp.leaf_cache.ptr) + cp.leaf[t].cache_off);
}

template <typename T>
int64_t put(std::vector<uint8_t>& blob, const std::vector<T>& v) {
  if (v.empty()) return -1;
  const int64_t off = align_up(static_cast<int64_t>(blob.size()));
  blob.resize(off + v.size() * sizeof(T));
  std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

}  // namespace

void materialize(const Net& net, ChunkPlan& cp, hipStream_t stream) {
  if (cp.materialized) return;
  std::vector<uint8_t>& blob = cp.host_blob;
  blob.clear();
  for (LeafPrep& lp : cp.leaf) {
    if (lp.direct || lp.inplace || !lp.perm.tiled) continue;
    PermuteHost& p = lp.perm;
    p.off_tile_in = put(blob, p.tile_in);
    p.off_slot_r = put(blob, p.tile_slot_r);
    p.off_tile_out = put(blob, p.tile_out);
    p.off_slot_w = put(blob, p.tile_slot_w);
    p.off_lo = put(blob, p.lo_tab);
    p.off_hi = put(blob, p.hi_tab);
  }
  for (StepPlan& sp : cp.steps) {
    if (sp.trans && sp.tperm.tiled) {
      PermuteHost& p = sp.tperm;
      p.off_tile_in = put(blob, p.tile_in);
      p.off_slot_r = put(blob, p.tile_slot_r);
      p.off_tile_out = put(blob, p.tile_out);
      p.off_slot_w = put(blob, p.tile_slot_w);
      p.off_lo = put(blob, p.lo_tab);
      p.off_hi = put(blob, p.hi_tab);
    }
    for (int q = 0; q < 4; ++q) sp.off_tab[q] = put(blob, sp.tab[q]);
    if (sp.offM.empty()) continue;
    sp.off_offM = put(blob, sp.offM);
    sp.off_offN = put(blob, sp.offN);
  }
  // grouped-launch tables reserve their space now and are filled once the
  // blob's device address (for the offset tables they point to) is known
  for (LevelPlan& L : cp.levels) {
    if (!L.group_steps.empty()) {
      L.off_gemm = put(blob, std::vector<GroupGemm>(L.group_steps.size()));
      L.off_gemm_prefix = put(blob, std::vector<int64_t>(L.group_steps.size()));
    }
    if (!L.group_leaves.empty()) {
      L.off_gather = put(blob, std::vector<GroupGather>(L.group_leaves.size()));
      L.off_gather_prefix = put(blob, std::vector<int64_t>(L.group_leaves.size()));
    }
  }
  if (!blob.empty()) cp.blob.alloc(blob.size());
  if (cp.cache_bytes) cp.leaf_cache.alloc(static_cast<size_t>(cp.cache_bytes));
  char* base = static_cast<char*>(cp.blob.ptr);
  for (StepPlan& sp : cp.steps) {
    const int64_t** tabs[4] = {&sp.desc.rowA, &sp.desc.kA, &sp.desc.rowB, &sp.desc.kB};
    for (int q = 0; q < 4; ++q)
      if (sp.off_tab[q] >= 0) *tabs[q] = reinterpret_cast<const int64_t*>(base + sp.off_tab[q]);
    if (sp.offM.empty()) continue;
    sp.dev_offM = reinterpret_cast<const int64_t*>(base + sp.off_offM);
    sp.dev_offN = reinterpret_cast<const int64_t*>(base + sp.off_offN);
    if (sp.split == 1) {  // the GEMM stores through them; else the split-K epilogue does
      sp.desc.offM = sp.dev_offM;
      sp.desc.offN = sp.dev_offN;
    }
  }
  const int n = net.n_tensors;
  for (LevelPlan& L : cp.levels) {
    if (!L.group_steps.empty()) {
      GroupGemm* tab = reinterpret_cast<GroupGemm*>(blob.data() + L.off_gemm);
      int64_t* pre = reinterpret_cast<int64_t*>(blob.data() + L.off_gemm_prefix);
      int64_t acc = 0;
      for (size_t q = 0; q < L.group_steps.size(); ++q) {
        const StepPlan& sp = cp.steps[L.group_steps[q]];
        GroupGemm g;
        std::memset(&g, 0, sizeof(g));
        g.d = sp.desc;
        auto operand = [&](int id, int32_t& rel) -> void* {
          if (id < n && (cp.leaf[id].direct || cp.leaf[id].inplace)) {
            rel = 0;
            return net.leaf[id].ptr;
          }
          if (id < n && cp.leaf[id].cached) {
            rel = 0;
            return cached_leaf(cp, id);
          }
          rel = 1;
          return reinterpret_cast<void*>(static_cast<intptr_t>(cp.buf_off[cp.tensor_buf[id]]));
        };
        g.d.A = static_cast<const float2*>(operand(sp.la, g.rel_a));
        g.d.B = static_cast<const float2*>(operand(sp.lb, g.rel_b));
        g.d.C = static_cast<float2*>(operand(sp.C, g.rel_c));
        g.slot_a = sp.la < n && cp.leaf[sp.la].inplace ? cp.leaf[sp.la].base_slot : -1;
        g.slot_b = sp.lb < n && cp.leaf[sp.lb].inplace ? cp.leaf[sp.lb].base_slot : -1;
        tab[q] = g;
        pre[q] = acc;
        acc += sp.desc.h * sp.desc.m * sp.desc.n;
      }
      L.gemm_total = acc;
    }
    if (!L.group_leaves.empty()) {
      GroupGather* tab = reinterpret_cast<GroupGather*>(blob.data() + L.off_gather);
      int64_t* pre = reinterpret_cast<int64_t*>(blob.data() + L.off_gather_prefix);
      int64_t acc = 0;
      for (size_t q = 0; q < L.group_leaves.size(); ++q) {
        const int t = L.group_leaves[q];
        const LeafPrep& lp = cp.leaf[t];
        GroupGather g;
        std::memset(&g, 0, sizeof(g));
        g.in = static_cast<const float2*>(net.leaf[t].ptr);
        g.out_off = cp.buf_off[cp.tensor_buf[t]];
        g.rank = lp.perm.plain.rank;
        g.base_slot = lp.base_slot;
        for (int r = 0; r < g.rank; ++r) {
          g.ext[r] = lp.perm.plain.ext[r];
          g.in_stride[r] = lp.perm.plain.in_stride[r];
        }
        tab[q] = g;
        pre[q] = acc;
        acc += cp.numel[t];
      }
      L.gather_total = acc;
    }
  }
  if (!blob.empty()) {
    // upload on the caller's stream and wait for it alone: other requests
    // keep running, and nobody sees the tables before they are complete
    check_hip(hipMemcpyAsync(cp.blob.ptr, blob.data(), blob.size(), hipMemcpyHostToDevice, stream),
              "upload plan tables");
    check_hip(hipStreamSynchronize(stream), "upload plan tables");
  }
  cp.materialized = true;
}

std::vector<std::pair<int, int64_t>> decompose(const Plan& plan, int64_t first, int64_t count) {
  std::vector<std::pair<int, int64_t>> out;
  int64_t s = first;
  const int64_t end = first + count;
  while (s < end) {
    int j = plan.j_max;
    while (j > 0 && (s % plan.suffix_prod[j] != 0 || s + plan.suffix_prod[j] > end)) --j;
    out.emplace_back(j, s);
    s += plan.suffix_prod[j];
  }
  return out;
}

namespace {

// Launch a planned gather-permute from `in` into `out` (tables in the chunk
// plan's device blob); `bd` points at a per-chunk base offset on the device
// (null: none).
hipError_t launch_planned_permute(const PermuteHost& p, const ChunkPlan& cp, const float2* in, float2* out,
                                  const int64_t* bd, hipStream_t stream, int planes = 0, int64_t pk = 0,
                                  int64_t pplane = 0) {
  const char* blob = static_cast<const char*>(cp.blob.ptr);
  if (p.tiled) {
    PermuteDesc d{};
    d.in = in;
    d.out = out;
    d.tile_in = reinterpret_cast<const int32_t*>(blob + p.off_tile_in);
    d.tile_slot_r = reinterpret_cast<const int32_t*>(blob + p.off_slot_r);
    d.tile_out = reinterpret_cast<const int32_t*>(blob + p.off_tile_out);
    d.tile_slot_w = reinterpret_cast<const int32_t*>(blob + p.off_slot_w);
    d.lo_tab = reinterpret_cast<const int64_t*>(blob + p.off_lo);
    d.hi_tab = reinterpret_cast<const int64_t*>(blob + p.off_hi);
    d.n_tiles = p.n_tiles;
    d.L = p.L;
    d.T = p.T;
    d.slots = p.slots;
    d.base = 0;
    d.base_dev = bd;
    d.pairs = p.pairs ? 1 : 0;
    d.planes = planes;
    d.pk = pk;
    d.pplane = pplane;
    return launch_permute(d, stream);
  }
  if (planes) return hipErrorInvalidValue;  // plane output is planned for tiled permutes only
  GatherDesc g = p.plain;
  g.in = in;
  g.out = out;
  g.base = 0;
  g.base_dev = bd;
  return launch_gather(g, stream);
}

// Launch the gather-permute of leaf t into `out`; `bd` points at its
// per-chunk base offset on the device (null: none).  planes = 1 / 2: out
// is the consuming step's A / B' planes (rows of pk complex).
hipError_t launch_leaf_prep(const Net& net, const ChunkPlan& cp, int t, float2* out, const int64_t* bd,
                            hipStream_t stream, int planes = 0, int64_t pk = 0, int64_t pplane = 0) {
  return launch_planned_permute(cp.leaf[t].perm, cp, static_cast<const float2*>(net.leaf[t].ptr), out, bd, stream,
                                planes, pk, pplane);
}

// (Re)fill the leaf cache when it is empty or a cached leaf's data has been
// replaced since.  Synchronous on `stream`; the context's stream is drained
// first so that leaf copies enqueued there have landed.
void refresh_leaf_cache(const Net& net, ChunkPlan& cp, hipStream_t stream) {
  if (!cp.n_cached) return;
  bool stale = cp.cache_version.empty();
  for (int t = 0; t < net.n_tensors && !stale; ++t)
    if (cp.leaf[t].cached && cp.cache_version[t] != net.version[t]) stale = true;
  if (!stale) return;
  if (stream != net.ctx->stream) check_hip(hipStreamSynchronize(net.ctx->stream), "leaf cache");
  for (int t = 0; t < net.n_tensors; ++t)
    if (cp.leaf[t].cached) check_hip(launch_leaf_prep(net, cp, t, cached_leaf(cp, t), nullptr, stream), "leaf cache");
  check_hip(hipStreamSynchronize(stream), "leaf cache");
  cp.cache_version = net.version;
}

ChunkPlan& ready(Plan& plan, int j, hipStream_t stream) {
  std::lock_guard<std::mutex> g(plan.mu);
  if (!plan.chunks[j]) plan.chunks[j] = build_chunk(plan, j);
  materialize(*plan.net, *plan.chunks[j], stream);
  refresh_leaf_cache(*plan.net, *plan.chunks[j], stream);
  return *plan.chunks[j];
}

struct Launcher {
  Plan& plan;
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>>* events;

  template <typename F>
  void run(int timer, hipStream_t stream, F&& f) {
    hipEvent_t a = nullptr, b = nullptr;
    if (events) {
      check_hip(hipEventCreate(&a), "event");
      check_hip(hipEventCreate(&b), "event");
      check_hip(hipEventRecord(a, stream), "event record");
    }
    check_hip(f(), "kernel launch");
    if (events) {
      check_hip(hipEventRecord(b, stream), "event record");
      events->push_back({{a, b}, timer});
    }
  }
};

}  // namespace

namespace {

// The launches of one chunk of one run, one piece at a time: a leaf's
// preparation, a step's GEMM, a level's grouped gathers and small GEMMs,
// the FP64 reduction of the root.  `bases` points at the chunk's leaf base
// offsets on the device.
struct ChunkOps {
  Plan& plan;
  ChunkPlan& cp;
  const RunArgs& a;
  const int64_t* bases;
  hipStream_t stream;
  Launcher& L;
  Net& net = *plan.net;
  const int n = net.n_tensors;
  const int ns = static_cast<int>(plan.pairs.size());
  const int t_prep = ns, t_red = ns + 1, t_group = ns + 2;
  const char* blob = static_cast<const char*>(cp.blob.ptr);
  const Form form = plan.form == TNC_GEMM_3M ? Form::M3 : Form::M4;
  const Prec prec = plan.prec == TNC_PREC_BF16X3 ? Prec::BF16X3 : Prec::C64;

  float2* ptr(int id) const {
    if (id < n && (cp.leaf[id].direct || cp.leaf[id].inplace)) return static_cast<float2*>(net.leaf[id].ptr);
    if (id < n && cp.leaf[id].cached) return cached_leaf(cp, id);
    if (id == cp.root_id && a.direct_out) return a.direct_out;
    return reinterpret_cast<float2*>(a.arena + cp.buf_off[cp.tensor_buf[id]]);
  }
  // a forced tile variant (tnc_ctx_set_gemm_variant) runs every MFMA step
  // on that variant, pre-split steps included
  bool presplit(const StepPlan& sp) const { return sp.presplit && net.ctx->gemm_variant < 0; }
  // 1 / 2: leaf t's permute writes its step's A / B' planes this run
  int planes_of(int t) const {
    const LeafPrep& lp = cp.leaf[t];
    return lp.planes_side && presplit(cp.steps[lp.step]) ? lp.planes_side : 0;
  }
  // the step's planes: A's, then B''s (in the 3M form each operand's r, i
  // and s planes)
  char* planes(const StepPlan& sp, int side) const {
    char* p = a.arena + cp.buf_off[sp.presplit_buf];
    if (form == Form::M3) return side == 2 ? p + presplit_3m_layout(sp.lm, sp.ln, sp.k).off_b : p;
    return side == 2 ? p + presplit_rows_a(sp.lm) * presplit_k(sp.k) * 8 : p;
  }
  void prep(int t) {
    const LeafPrep& lp = cp.leaf[t];
    const int side = planes_of(t);
    const StepPlan* sp = side ? &cp.steps[lp.step] : nullptr;
    float2* out = side ? reinterpret_cast<float2*>(planes(*sp, side)) : ptr(t);
    const int64_t* bd = lp.base_slot >= 0 ? bases + lp.base_slot : nullptr;
    const int64_t pk = side ? sp->k : 0;
    // 3M form: one plane mode for both operands, planes of padded rows x k
    int mode = side;
    int64_t pplane = 0;
    if (side && form == Form::M3) {
      const Presplit3M g = presplit_3m_layout(sp->lm, sp->ln, sp->k);
      mode = 3;
      pplane = (side == 1 ? g.mp : g.np) * 2 * g.kp;
    }
    L.run(t_prep, stream, [&] { return launch_leaf_prep(net, cp, t, out, bd, stream, mode, pk, pplane); });
  }
  int variant(const StepPlan& sp) const { return net.ctx->gemm_variant >= 0 ? net.ctx->gemm_variant : sp.variant; }
  // The step's launch descriptor with this run's pointers (the split-K
  // partials, or the output before its separate transpose, go to the
  // step's arena scratch buffer).
  GemmDesc desc(int s) const {
    const StepPlan& sp = cp.steps[s];
    GemmDesc d = sp.desc;
    d.A = ptr(sp.la);
    d.B = ptr(sp.lb);
    d.C = sp.split > 1 || sp.trans ? reinterpret_cast<float2*>(a.arena + cp.buf_off[sp.scratch_buf]) : ptr(sp.C);
    auto slot = [&](int id) { return id < n && cp.leaf[id].inplace ? bases + cp.leaf[id].base_slot : nullptr; };
    d.baseA = slot(sp.la);
    d.baseB = slot(sp.lb);
    return d;
  }
  // What follows the GEMM: the split-K epilogue, or the separate transpose
  // into the consumer's order.
  void finish(int s) {
    const StepPlan& sp = cp.steps[s];
    if (sp.split <= 1 && !sp.trans) return;
    const GemmDesc d = desc(s);
    float2* c = ptr(sp.C);
    if (sp.trans) {
      L.run(s, stream, [&] { return launch_planned_permute(sp.tperm, cp, d.C, c, nullptr, stream); });
      return;
    }
    L.run(s, stream, [&] {
      return launch_splitk_reduce(d.C, c, sp.h, sp.lm, sp.ln, sp.split, sp.dev_offM, sp.dev_offN, stream);
    });
  }
  void step(int s) {
    const StepPlan& sp = cp.steps[s];
    const GemmDesc d = desc(s);
    if (presplit(sp) && form == Form::M3) {
      void* p = planes(sp, 1);
      const bool have_a = sp.la < n && planes_of(sp.la) == 1, have_b = sp.lb < n && planes_of(sp.lb) == 2;
      L.run(s, stream, [&] { return launch_gemm_presplit_3m(d, p, have_a, have_b, stream); });
    } else if (presplit(sp)) {
      void* p = planes(sp, 1);
      // operands whose permute wrote the planes are not split again
      const bool have_a = sp.la < n && planes_of(sp.la) == 1, have_b = sp.lb < n && planes_of(sp.lb) == 2;
      L.run(s, stream, [&] { return launch_gemm_presplit(d, p, have_a, have_b, stream); });
    } else {
      L.run(s, stream, [&] { return launch_gemm(d, sp.kind, variant(sp), form, prec, stream); });
    }
    finish(s);
  }
  void level_gathers(const LevelPlan& lv) {
    if (lv.group_leaves.empty()) return;
    L.run(t_prep, stream, [&] {
      return launch_group_gather(reinterpret_cast<const GroupGather*>(blob + lv.off_gather),
                                 reinterpret_cast<const int64_t*>(blob + lv.off_gather_prefix),
                                 static_cast<int>(lv.group_leaves.size()), lv.gather_total, a.arena, bases, stream);
    });
  }
  void level_small_gemms(const LevelPlan& lv) {
    if (lv.group_steps.empty()) return;
    L.run(t_group, stream, [&] {
      return launch_group_gemm(reinterpret_cast<const GroupGemm*>(blob + lv.off_gemm),
                               reinterpret_cast<const int64_t*>(blob + lv.off_gemm_prefix),
                               static_cast<int>(lv.group_steps.size()), lv.gemm_total, a.arena, bases, prec, stream);
    });
  }
  void reduce(bool overwrite) {
    if (a.direct_out) return;
    const float2* root = ptr(cp.root_id);
    L.run(t_red, stream, [&] { return launch_reduce_fp64(root, a.acc, cp.hs, cp.R, overwrite, stream); });
  }
};

// Enqueue one chunk: leaf permutations, one GEMM per step, the FP64
// reduction of the root.  `bases` points at this chunk's leaf base offsets.
void enqueue_chunk(Plan& plan, ChunkPlan& cp, const RunArgs& a, const int64_t* bases, bool overwrite,
                   hipStream_t stream, Launcher& L) {
  ChunkOps op{plan, cp, a, bases, stream, L};
  if (op.ns == 0 && !cp.leaf[0].direct) op.prep(0);
  if (cp.grouped) {
    // level by level: the level's plain leaf gathers in one launch, its small
    // GEMMs in another, everything else one launch each
    for (const LevelPlan& lv : cp.levels) {
      op.level_gathers(lv);
      for (int t : lv.single_leaves) op.prep(t);
      op.level_small_gemms(lv);
      for (int s : lv.single_steps) op.step(s);
    }
  } else {
    for (int s = 0; s < op.ns; ++s) {
      for (int t : cp.steps[s].preps) op.prep(t);
      op.step(s);
    }
  }
  op.reduce(overwrite);
}

// The captured graph of one chunk plan for one set of buffers (created on
// first use, replayed afterwards), or nullptr once the plan holds
// kMaxGraphsPerPlan graphs: callers that keep handing in new buffers (a new
// output tensor per call, requests at ever different arena offsets) then run
// the chunk eagerly instead of growing the cache.  Nothing is evicted, so no
// graph is destroyed while another thread may have it in flight.
constexpr size_t kMaxGraphsPerPlan = 64;

hipGraphExec_t chunk_graph(Plan& plan, ChunkPlan& cp, const RunArgs& a, const int64_t* cur_bases, bool overwrite) {
  const GraphKey key{cp.j, a.arena, a.acc, a.direct_out, cur_bases, overwrite, plan.net->ctx->gemm_variant};
  std::lock_guard<std::mutex> g(plan.graph_mu);
  auto it = plan.graphs.find(key);
  if (it != plan.graphs.end()) return it->second;
  if (plan.graphs.size() >= kMaxGraphsPerPlan) return nullptr;
  // capture and instantiation run alone in the process (runtime_mu)
  std::lock_guard<std::recursive_mutex> rt(runtime_mu());
  if (!plan.capture_stream) check_hip(hipStreamCreate(&plan.capture_stream), "hipStreamCreate");
  hipGraph_t graph = nullptr;
  check_hip(hipStreamBeginCapture(plan.capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  Launcher none{plan, nullptr};
  try {
    enqueue_chunk(plan, cp, a, cur_bases, overwrite, plan.capture_stream, none);
  } catch (...) {
    (void)hipStreamEndCapture(plan.capture_stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  check_hip(hipStreamEndCapture(plan.capture_stream, &graph), "end capture");
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  check_hip(e, "graph instantiate");
  plan.graphs.emplace(key, exec);
  return exec;
}

}  // namespace

// Add the timings of profiled launches to the step timers and free their
// events (plan.mu held): all of them, waiting for each, or only those that
// have completed.
static void fold_events(Plan& plan, bool wait) {
  size_t keep = 0;
  for (size_t i = 0; i < plan.pending.size(); ++i) {
    const auto e = plan.pending[i];
    if (wait)
      check_hip(hipEventSynchronize(e.first.second), "event sync");
    else if (hipEventQuery(e.first.second) != hipSuccess) {
      plan.pending[keep++] = e;
      continue;
    }
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, e.first.first, e.first.second), "event time");
    StepTimer& t = plan.timers[e.second];
    t.ms += ms;
    t.launches += 1;
    (void)hipEventDestroy(e.first.first);
    (void)hipEventDestroy(e.first.second);
  }
  plan.pending.resize(keep);
}

int64_t run_workspace_bytes(Plan& plan, int64_t first, int64_t count) {
  const auto chunks = decompose(plan, first, count);
  int64_t peak = 0;
  int slots = 1;
  for (auto& c : chunks) {
    ChunkPlan& cp = plan.chunk(c.first);
    peak = std::max(peak, cp.peak);
    slots = std::max(slots, cp.n_base_slots);
  }
  return align_up(peak) + align_up(slots * 8) + align_up(static_cast<int64_t>(chunks.size()) * slots * 8);
}

namespace {

// The chunks of a run, every chunk plan ready on the device, and the
// per-chunk leaf base offsets uploaded into the run's workspace
// ([intermediates | current chunk's bases | all chunks' bases]).
struct RunBases {
  std::vector<std::pair<int, int64_t>> chunks;
  int slots = 1;
  int64_t* cur_dev = nullptr;
  int64_t* bases_dev = nullptr;
};

RunBases prepare_run(Plan& plan, const RunArgs& a) {
  Net& net = *plan.net;
  RunBases rb;
  rb.chunks = decompose(plan, a.first, a.count);
  const auto& chunks = rb.chunks;
  if (chunks.empty()) fail(TNC_E_ARG, "empty slice range");
  // per-chunk base offsets of leaves that carry fixed sliced labels
  int slots = 1;
  for (auto& c : chunks) slots = std::max(slots, ready(plan, c.first, a.stream).n_base_slots);
  const int64_t nS = static_cast<int64_t>(plan.sliced.size());
  std::vector<int64_t> bases(chunks.size() * slots, 0);
  int64_t peak = 0;
  for (size_t c = 0; c < chunks.size(); ++c) {
    ChunkPlan& cp = ready(plan, chunks[c].first, a.stream);
    peak = std::max(peak, cp.peak);
    if (!cp.n_base_slots) continue;
    std::vector<int64_t> val(net.extents.size(), 0);
    int64_t rest = chunks[c].second;
    for (int64_t q = nS - 1; q >= 0; --q) {
      const int l = plan.sliced[q];
      val[l] = rest % net.extents[l];
      rest /= net.extents[l];
    }
    for (const LeafPrep& lp : cp.leaf) {
      if (lp.base_slot < 0) continue;
      int64_t off = 0;
      for (auto& f : lp.fixed) off += val[f.first] * f.second;
      bases[c * slots + lp.base_slot] = off;
    }
  }
  const int64_t cur_off = align_up(peak);
  const int64_t bases_off = cur_off + align_up(slots * 8);
  const size_t need = static_cast<size_t>(bases_off) + bases.size() * sizeof(int64_t);
  if (need > a.arena_bytes)
    fail(TNC_E_NOMEM, "run needs " + std::to_string(need) + " arena bytes, have " + std::to_string(a.arena_bytes));
  rb.slots = slots;
  rb.cur_dev = reinterpret_cast<int64_t*>(a.arena + cur_off);
  rb.bases_dev = reinterpret_cast<int64_t*>(a.arena + bases_off);
  // leaves with fixed sliced labels read their per-chunk offsets on the
  // device; without any, nothing needs uploading (or copying per chunk).
  // The host vector is pageable: the runtime copies it before returning.
  bool any_bases = false;
  for (auto& c : chunks) any_bases |= plan.chunks[c.first]->n_base_slots > 0;
  if (any_bases)
    check_hip(hipMemcpyAsync(rb.bases_dev, bases.data(), bases.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                             a.stream),
              "upload chunk bases");
  return rb;
}

}  // namespace

void run_plan(Plan& plan, const RunArgs& a) {
  const int ns = static_cast<int>(plan.pairs.size());
  const RunBases rb = prepare_run(plan, a);
  const auto& chunks = rb.chunks;
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> ev;
  Launcher L{plan, plan.profile && !plan.graph ? &ev : nullptr};
  for (size_t c = 0; c < chunks.size(); ++c) {
    ChunkPlan& cp = ready(plan, chunks[c].first, a.stream);
    hipGraphExec_t exec = plan.graph ? chunk_graph(plan, cp, a, rb.cur_dev, a.fresh_acc && c == 0) : nullptr;
    if (exec) {
      if (cp.n_base_slots)
        check_hip(hipMemcpyAsync(rb.cur_dev, rb.bases_dev + c * rb.slots, rb.slots * sizeof(int64_t),
                                 hipMemcpyDeviceToDevice, a.stream),
                  "chunk bases");
      check_hip(hipGraphLaunch(exec, a.stream), "graph launch");
    } else {
      enqueue_chunk(plan, cp, a, rb.bases_dev + c * rb.slots, a.fresh_acc && c == 0, a.stream, L);
    }
  }
  if (!ev.empty()) {
    std::lock_guard<std::mutex> g(plan.mu);
    if (plan.timers.size() < static_cast<size_t>(ns + 3)) plan.timers.resize(ns + 3);
    for (auto& e : ev) plan.pending.push_back(e);
    // long profiled sessions: fold what has finished without waiting
    if (plan.pending.size() > 16384) fold_events(plan, false);
  }
}

// ------------------------------------------------------------------ lockstep
// Several runs of plans with one structure (the same path, shapes, chunking
// and tile variants, see structure_key) over slice ranges with the same
// chunk sequence, executed together on one stream: chunk by chunk and level
// by level, every run's leaf preparations and small GEMMs are launched as
// in a run of its own, and every MFMA step goes out as one grouped launch
// over the runs' GEMMs of that step.  Each output element is computed by the
// same tile code in the same order as alone, so every run's result is
// bitwise its result alone.

std::string structure_key(Plan& plan, int64_t first, int64_t count) {
  std::string k;
  auto put = [&](int64_t v) { k.append(reinterpret_cast<const char*>(&v), sizeof v); };
  {
    // what a plan fixes at creation (network shape, path, slicing) is keyed
    // once per plan
    std::lock_guard<std::mutex> g(plan.mu);
    if (plan.key_prefix.empty()) {
      const Net& net = *plan.net;
      put(net.n_tensors);
      for (const auto& lab : net.labels) {
        put(static_cast<int64_t>(lab.size()));
        for (int l : lab) put(l);
      }
      put(static_cast<int64_t>(net.extents.size()));
      for (int64_t e : net.extents) put(e);
      put(static_cast<int64_t>(net.open.size()));
      for (int l : net.open) put(l);
      for (const auto& pr : plan.pairs) put(pr[0] * int64_t{1 << 30} + pr[1]);
      put(static_cast<int64_t>(plan.sliced.size()));
      for (int l : plan.sliced) put(l);
      plan.key_prefix = k;
    }
    k = plan.key_prefix;
  }
  put(plan.prec);
  put(plan.form);
  put(plan.grouping);
  put(plan.store_order);
  put(plan.net->ctx->gemm_variant);
  put(static_cast<int64_t>(plan.volatile_leaf.size()));
  for (char v : plan.volatile_leaf) put(v);
  const auto chunks = decompose(plan, first, count);
  put(static_cast<int64_t>(chunks.size()));
  std::vector<char> seen(plan.chunks.size(), 0);
  for (auto& c : chunks) {
    put(c.first);
    if (seen[c.first]) continue;
    seen[c.first] = 1;
    const ChunkPlan& cp = plan.chunk(c.first);
    for (const StepPlan& sp : cp.steps) {
      put(static_cast<int64_t>(sp.kind));
      put(sp.variant);
      put(sp.split);
    }
  }
  return k;
}

namespace {

constexpr size_t kTableAlign = 256;
size_t table_align(size_t x) { return (x + kTableAlign - 1) / kTableAlign * kTableAlign; }

}  // namespace

LockstepInfo lockstep_info(Plan& plan, int64_t first, int64_t count) {
  LockstepInfo t;
  const auto chunks = decompose(plan, first, count);
  std::vector<char> seen(plan.chunks.size(), 0);
  for (auto& c : chunks) {
    const ChunkPlan& cp = plan.chunk(c.first);
    // launches of this chunk in a run of its own (enqueue_chunk's order)
    auto step_launches = [&](const StepPlan& sp) { return 1 + (sp.split > 1 || sp.trans ? 1 : 0); };
    int64_t nl = 1 + (cp.n_base_slots ? 1 : 0);  // reduction, chunk bases
    if (cp.steps.empty() && !cp.leaf[0].direct) ++nl;
    if (cp.grouped) {
      for (const LevelPlan& lv : cp.levels) {
        nl += (lv.group_leaves.empty() ? 0 : 1) + (lv.group_steps.empty() ? 0 : 1);
        nl += static_cast<int64_t>(lv.single_leaves.size());
        for (int s : lv.single_steps) nl += step_launches(cp.steps[s]);
      }
    } else {
      for (const StepPlan& sp : cp.steps) nl += static_cast<int64_t>(sp.preps.size()) + step_launches(sp);
    }
    t.launches += nl;
    if (seen[c.first]) continue;
    seen[c.first] = 1;
    for (const StepPlan& sp : cp.steps)
      if (sp.kind == GemmKernel::MFMA) {
        t.bytes_per_run += sizeof(GroupedEntry);
        t.parts += 1;
      }
    if (!cp.grouped) continue;
    for (const LevelPlan& lv : cp.levels) {  // per run: one GroupRun per grouped launch
      if (!lv.group_steps.empty()) {
        t.bytes_per_run += sizeof(GroupRun);
        t.parts += 1;
      }
      if (!lv.group_leaves.empty()) {
        t.bytes_per_run += sizeof(GroupRun);
        t.parts += 1;
      }
    }
  }
  return t;
}

size_t lockstep_table_bytes(const LockstepInfo& t, int n_runs) {
  return static_cast<size_t>(n_runs) * t.bytes_per_run + static_cast<size_t>(t.parts) * kTableAlign + kTableAlign;
}

void run_lockstep(std::vector<LockstepRun>& runs, void* host_tables, void* dev_tables, size_t cap,
                  hipStream_t stream) {
  const int K = static_cast<int>(runs.size());
  if (K < 1) return;
  std::vector<RunBases> rb;
  for (auto& r : runs) rb.push_back(prepare_run(*r.plan, r.a));
  for (int r = 1; r < K; ++r) {
    bool same = rb[r].chunks.size() == rb[0].chunks.size();
    for (size_t c = 0; same && c < rb[0].chunks.size(); ++c) same = rb[r].chunks[c].first == rb[0].chunks[c].first;
    if (!same) fail(TNC_E_ARG, "lockstep runs need the same chunk sequence");
  }
  Plan& p0 = *runs[0].plan;
  const Form form = p0.form == TNC_GEMM_3M ? Form::M3 : Form::M4;
  const Prec prec = p0.prec == TNC_PREC_BF16X3 ? Prec::BF16X3 : Prec::C64;
  Launcher none{p0, nullptr};
  auto ops_of = [&](size_t c) {
    std::vector<std::unique_ptr<ChunkOps>> ops;
    const int j = rb[0].chunks[c].first;
    for (int r = 0; r < K; ++r)
      ops.emplace_back(new ChunkOps{*runs[r].plan, *runs[r].plan->chunks[j], runs[r].a, rb[r].cur_dev, stream, none});
    return ops;
  };
  // Tables of the job, built once on the host and uploaded once: per MFMA
  // step the K runs' GEMMs (grouped launch), per tree level one GroupRun
  // per run for its small GEMMs and one for its plain gathers.  Tables
  // serve every chunk of a chunk plan, so leaf bases are read from each
  // run's "current chunk" slot, refreshed before the chunk's first launch.
  char* host = static_cast<char*>(host_tables);
  char* dev = static_cast<char*>(dev_tables);
  size_t used = 0;
  auto take = [&](size_t bytes) -> size_t {
    const size_t off = table_align(used);
    if (off + bytes > cap) fail(TNC_E_NOMEM, "grouped-launch tables exceed their buffer");
    used = off + bytes;
    return off;
  };
  struct LevelTabs {
    size_t gemm = 0, gath = 0;   // offsets of the GroupRun tables
    int n_gemm = 0, n_gath = 0;  // runs in them (0: no such launch)
    int64_t gemm_total = 0, gath_total = 0;
  };
  std::map<std::pair<int, int>, std::pair<size_t, int64_t>> grouped;  // (j, step) -> (offset, tiles)
  std::map<std::pair<int, int>, LevelTabs> levtabs;                   // (j, level)
  std::vector<char> built(p0.chunks.size(), 0);
  for (size_t c = 0; c < rb[0].chunks.size(); ++c) {
    const int j = rb[0].chunks[c].first;
    if (built[j]) continue;
    built[j] = 1;
    const ChunkPlan& cp0 = *p0.chunks[j];
    auto ops = ops_of(c);
    for (int s = 0; s < static_cast<int>(cp0.steps.size()); ++s) {
      if (cp0.steps[s].kind != GemmKernel::MFMA || ops[0]->presplit(cp0.steps[s])) continue;
      const int v = ops[0]->variant(cp0.steps[s]);
      if (!grouped_variant_ok(form, prec, v)) continue;  // no grouped form: per-request launches
      bool ok = true;
      for (int r = 0; ok && r < K; ++r) {
        const StepPlan& sp = ops[r]->cp.steps[s];
        ok = sp.kind == GemmKernel::MFMA && ops[r]->variant(sp) == v;
      }
      if (!ok) continue;
      const size_t off = take(K * sizeof(GroupedEntry));
      auto* e = reinterpret_cast<GroupedEntry*>(host + off);
      for (int r = 0; r < K; ++r) {
        std::memset(&e[r], 0, sizeof(GroupedEntry));
        e[r].d = ops[r]->desc(s);
      }
      const int64_t total = grouped_layout(e, K, v);
      if (total > 0) grouped[{j, s}] = {off, total};
    }
    if (!cp0.grouped) continue;
    // per level, the runs' own device tables (materialized with each plan)
    // as one launch over runs: each run brings its arena and its current
    // leaf bases, so no run's table is copied or rewritten here
    for (size_t li = 0; li < cp0.levels.size(); ++li) {
      LevelTabs t;
      const LevelPlan& lv0 = cp0.levels[li];
      auto runs_table = [&](bool gemm_tab, int64_t& total) {
        const size_t off = take(K * sizeof(GroupRun));
        auto* gr = reinterpret_cast<GroupRun*>(host + off);
        for (int r = 0; r < K; ++r) {
          const ChunkPlan& cp = ops[r]->cp;
          const LevelPlan& lv = cp.levels[li];
          const char* blob = static_cast<const char*>(cp.blob.ptr);
          std::memset(&gr[r], 0, sizeof(GroupRun));
          gr[r].table = blob + (gemm_tab ? lv.off_gemm : lv.off_gather);
          gr[r].prefix = reinterpret_cast<const int64_t*>(blob + (gemm_tab ? lv.off_gemm_prefix : lv.off_gather_prefix));
          gr[r].n = static_cast<int32_t>(gemm_tab ? lv.group_steps.size() : lv.group_leaves.size());
          gr[r].arena = runs[r].a.arena;
          gr[r].bases = rb[r].cur_dev;
          gr[r].first = total;
          total += gemm_tab ? lv.gemm_total : lv.gather_total;
        }
        return off;
      };
      if (!lv0.group_steps.empty()) {
        t.n_gemm = K;
        t.gemm = runs_table(true, t.gemm_total);
      }
      if (!lv0.group_leaves.empty()) {
        t.n_gath = K;
        t.gath = runs_table(false, t.gath_total);
      }
      levtabs[{j, static_cast<int>(li)}] = t;
    }
  }
  if (used)
    check_hip(hipMemcpyAsync(dev, host, used, hipMemcpyHostToDevice, stream), "upload grouped tables");
  for (size_t c = 0; c < rb[0].chunks.size(); ++c) {
    const int j = rb[0].chunks[c].first;
    auto ops = ops_of(c);
    const ChunkPlan& cp0 = *p0.chunks[j];
    for (int r = 0; r < K; ++r)  // the chunk's leaf bases into each run's current slot
      if (ops[r]->cp.n_base_slots)
        check_hip(hipMemcpyAsync(rb[r].cur_dev, rb[r].bases_dev + c * rb[r].slots, rb[r].slots * sizeof(int64_t),
                                 hipMemcpyDeviceToDevice, stream),
                  "chunk bases");
    auto gemm = [&](int s) {
      auto it = grouped.find({j, s});
      if (it == grouped.end()) {
        for (auto& op : ops) op->step(s);
        return;
      }
      const int v = ops[0]->variant(cp0.steps[s]);
      check_hip(launch_gemm_grouped(reinterpret_cast<const GroupedEntry*>(dev + it->second.first), K,
                                    it->second.second, v, form, prec, stream),
                "grouped GEMM launch");
      for (auto& op : ops) op->finish(s);
    };
    const int ns = static_cast<int>(cp0.steps.size());
    if (ns == 0)
      for (auto& op : ops)
        if (!op->cp.leaf[0].direct) op->prep(0);
    if (cp0.grouped) {
      for (size_t li = 0; li < cp0.levels.size(); ++li) {
        const LevelTabs& t = levtabs.at({j, static_cast<int>(li)});
        if (t.n_gath)
          check_hip(launch_group_gather_runs(reinterpret_cast<const GroupRun*>(dev + t.gath), t.n_gath, t.gath_total,
                                             stream),
                    "grouped gathers");
        for (auto& op : ops)
          for (int tl : op->cp.levels[li].single_leaves) op->prep(tl);
        if (t.n_gemm)
          check_hip(launch_group_gemm_runs(reinterpret_cast<const GroupRun*>(dev + t.gemm), t.n_gemm, t.gemm_total,
                                           prec, stream),
                    "grouped small GEMMs");
        for (int s : cp0.levels[li].single_steps) gemm(s);
      }
    } else {
      for (int s = 0; s < ns; ++s) {
        for (auto& op : ops)
          for (int tl : op->cp.steps[s].preps) op->prep(tl);
        gemm(s);
      }
    }
    for (int r = 0; r < K; ++r) ops[r]->reduce(runs[r].a.fresh_acc && c == 0);
  }
}

Plan::~Plan() {
  if (net && !net->ctx->host_only) {
    (void)hipSetDevice(net->ctx->device);
    (void)hipStreamSynchronize(net->ctx->stream);
  }
  for (auto& e : pending) {
    (void)hipEventDestroy(e.first.first);
    (void)hipEventDestroy(e.first.second);
  }
  std::lock_guard<std::recursive_mutex> rt(runtime_mu());
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  pinned_free(host_res);
  chunks.clear();  // device tables and leaf caches, freed under the lock
  acc.reset();
  norm.reset();
}

void Plan::drop_graphs() {
  const Ctx& c = *net->ctx;
  if (!c.host_only) check_hip(hipStreamSynchronize(c.stream), "sync before dropping graphs");
  std::lock_guard<std::mutex> lk(graph_mu);
  std::lock_guard<std::recursive_mutex> rt(runtime_mu());
  for (auto& e : graphs) (void)hipGraphExecDestroy(e.second);
  graphs.clear();
}

void drain_profile(Plan& plan) {
  std::lock_guard<std::mutex> g(plan.mu);
  fold_events(plan, true);
}

}  // namespace tnc
