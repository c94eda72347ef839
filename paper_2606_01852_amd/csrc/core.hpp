// Host-side structures of the path executor (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <map>
#include <cstdint>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tnc.h"
#include "kernels.hpp"

namespace tnc {

// Error carrying a status code; caught at the ABI boundary.
struct Error {
  tnc_status code;
  std::string msg;
};
[[noreturn]] void fail(tnc_status code, const std::string& msg);
void check_hip(hipError_t e, const char* what);
struct Ctx;
void set_device(const Ctx& c);
void g_error_clear();
void g_error_set(const std::string& m);
const char* g_error_get();

// Process-wide lock around the HIP runtime calls that capture, allocate or
// free: graph capture and instantiation, graph destruction, device and
// pinned host allocations and frees, stream creation and destruction.
// Server workers of every context capture graphs and grow staging buffers
// from their own threads; with this lock no allocation or free (some of
// which synchronise the device) runs while another thread is between the
// begin and the end of a capture, and no two captures overlap, so nothing
// depends on how the runtime handles such overlaps.  Recursive: a holder
// may allocate.
std::recursive_mutex& runtime_mu();
// Pinned host memory (hipHostMalloc / hipHostFree) under runtime_mu().
void* pinned_alloc(size_t bytes, const char* what);
void pinned_free(void* p);

// Device allocation owned by the library.
struct DeviceBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DeviceBuf() = default;
  DeviceBuf(const DeviceBuf&) = delete;
  DeviceBuf& operator=(const DeviceBuf&) = delete;
  DeviceBuf(DeviceBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes) {
    o.ptr = nullptr;
    o.bytes = 0;
  }
  ~DeviceBuf();
  void alloc(size_t n);
  void reset();
};

struct Server;

// Autotuning key: one GEMM step shape.
struct TuneKey {
  int prec = 0, form = 0, perm = 0;
  int64_t h = 0, m = 0, n = 0, k = 0;
  bool operator<(const TuneKey& o) const {
    if (prec != o.prec) return prec < o.prec;
    if (form != o.form) return form < o.form;
    if (perm != o.perm) return perm < o.perm;
    if (h != o.h) return h < o.h;
    if (m != o.m) return m < o.m;
    if (n != o.n) return n < o.n;
    return k < o.k;
  }
  std::string str() const;
};

struct Ctx {
  int device = -1;
  bool host_only = true;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  bool own_arena = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DeviceBuf scratch;   // tables of stand-alone permutes
  int gemm_variant = -1; // forced MFMA tile variant (-1: autotuned / default)
  std::mutex tune_mu;
  std::map<TuneKey, int> tune_cache;  // autotuned tile variant per step shape
  std::shared_ptr<Server> server;
  ~Ctx();
};

enum class LabelKind : uint8_t { Unused = 0, Closed, Open, Batch };

struct Net {
  std::shared_ptr<Ctx> ctx_ref;           // keeps the context alive (destroyed last)
  Ctx* ctx = nullptr;
  int n_tensors = 0;
  std::vector<std::vector<int>> labels;   // stored order per leaf
  std::vector<int64_t> extents;           // per label
  std::vector<int> open;                  // result order
  std::vector<LabelKind> kind;            // per label
  std::vector<int> user_batch;            // batch labels in open order
  std::vector<int64_t> numel;             // per leaf
  std::vector<DeviceBuf> leaf;            // resident complex64 leaves
  std::vector<uint64_t> version;          // per leaf, bumped when its data is replaced
  std::atomic<int> n_batchers{0};         // a batcher writes rows of its leaves
  std::vector<std::vector<int64_t>> stride;  // per leaf, per stored mode
  ~Net();
};

// A tile decomposition of one gather-permute (host copy of the tables).
struct PermuteHost {
  bool tiled = false;
  // every even read-order element and its successor are adjacent in the
  // input, every even write-order element and its successor adjacent in the
  // output, all at even offsets: the tile moves as 16-byte pairs
  bool pairs = false;
  int32_t T = 0, slots = 0, L = 1;
  int64_t n_tiles = 0;
  std::vector<int32_t> tile_in, tile_slot_r, tile_out, tile_slot_w;
  std::vector<int64_t> lo_tab, hi_tab;
  GatherDesc plain{};
  // offsets of the tables inside the plan's device blob
  int64_t off_tile_in = -1, off_slot_r = -1, off_tile_out = -1, off_slot_w = -1, off_lo = -1, off_hi = -1;
};

// Build the gather-permute out[w] = in[base + sum_d digit_d(w) * in_stride[d]]
// for row-major output dims ext[].
PermuteHost build_permute(const std::vector<int64_t>& ext, const std::vector<int64_t>& in_stride);

struct LeafPrep {
  int leaf = -1;
  bool direct = true;        // use the resident leaf as is
  int buf = -1;              // arena buffer when prepared
  int base_slot = -1;        // slot of its per-chunk base offset (-1: none)
  std::vector<std::pair<int, int64_t>> fixed;  // (sliced label, stride) fixed per chunk
  PermuteHost perm;
  int step = -1;             // step that consumes it
  // a leaf with no per-chunk base offset is permuted once into the chunk
  // plan's leaf cache (refreshed when its data is replaced), not per run
  bool cached = false;
  int64_t cache_off = -1;
  // a leaf with a per-chunk base offset consumed by a one-thread-per-output
  // GEMM is read in place through the step's operand tables (no gather)
  bool inplace = false;
  // a tiled permute feeding a pre-split step writes that step's planes
  // (1: its A, 2: its B') instead of complex64, when the step runs pre-split
  int planes_side = 0;
};

struct StepPlan {
  int A = -1, B = -1, C = -1;                 // tensor ids (A = M side)
  std::vector<int> H, M, N, K;
  int64_t h = 1, m = 1, n = 1, k = 1, hA = 1, hB = 1;
  bool natural = true;
  // launch: the GEMM may run transposed (B as the row operand) when that
  // fills MFMA tiles better, and with K split into `split` parts whose
  // partial products go to an arena scratch buffer and are summed by the
  // split-K epilogue
  bool swap = false;
  int la = -1, lb = -1;                       // launch operands (row, column)
  int64_t lm = 1, ln = 1;                     // launch rows / columns
  int split = 1;
  int scratch_buf = -1;                       // arena buffer of the partials
  GemmKernel kind = GemmKernel::SMALL;
  int variant = 0;                            // MFMA tile variant (autotuned)
  GemmDesc desc{};                            // launch descriptor; pointers filled at run time
  int64_t off_offM = -1, off_offN = -1;       // in the device blob
  std::vector<int64_t> offM, offN;            // store tables in launch orientation (empty: natural)
  const int64_t* dev_offM = nullptr;          // device copies of the store tables
  const int64_t* dev_offN = nullptr;
  std::vector<int> preps;                     // leaf preps launched before the GEMM
  // separate-transpose store (the plan's store order 1): the GEMM stores
  // [H | launch rows | launch columns] into the step's scratch buffer and
  // this permutation writes it in the consumer's order
  bool trans = false;
  PermuteHost tperm;
  // split precision on operands split once into bf16 planes (large steps of
  // one batch entry): the planes live in this arena buffer during the step
  bool presplit = false;
  int presplit_buf = -1;
  // in-place operand tables (launch orientation): rowA, kA, rowB, kB
  std::vector<int64_t> tab[4];
  int64_t off_tab[4] = {-1, -1, -1, -1};
};

// One level of the contraction tree: the steps whose operands are all
// produced at lower levels.  Small steps and plain leaf gathers of a level
// run as one grouped launch each; MFMA/long-K steps and tiled permutes run
// alone.
struct LevelPlan {
  std::vector<int> group_leaves, single_leaves;
  std::vector<int> group_steps, single_steps;
  int64_t off_gemm = -1, off_gemm_prefix = -1, gemm_total = 0;
  int64_t off_gather = -1, off_gather_prefix = -1, gather_total = 0;
};

struct ChunkPlan {
  int j = 0;                       // number of trailing sliced labels batched
  bool grouped = false;            // execute level by level
  std::vector<LevelPlan> levels;
  int64_t hs = 1;                  // slices per chunk
  std::vector<int> batch;          // canonical batch labels
  std::vector<std::vector<int>> order;   // per tensor id
  std::vector<int64_t> numel;            // per tensor id
  std::vector<LeafPrep> leaf;            // per leaf
  std::vector<StepPlan> steps;
  std::vector<int64_t> buf_bytes, buf_off;  // arena buffers
  std::vector<int> tensor_buf;              // per tensor id: arena buffer or -1
  int64_t peak = 0;                          // arena bytes
  int root_id = -1;
  int64_t R = 1;                             // result elements
  int n_base_slots = 0;
  std::vector<int64_t> result_perm;          // user index -> reduced-root index
  // device side (built on first use)
  bool materialized = false;
  DeviceBuf blob;
  DeviceBuf leaf_cache;                      // permuted copies of the cached leaves
  int64_t cache_bytes = 0;
  int n_cached = 0;
  std::vector<uint64_t> cache_version;       // leaf versions the cache holds (empty: not filled)
  std::vector<uint8_t> host_blob;
  double flops = 0, bytes = 0, transpose_bytes = 0;
  int64_t max_tensor = 0;
  int n_permutes = 0, n_perm_stores = 0;
};

struct StepTimer {
  double ms = 0;
  int64_t launches = 0;
};

struct GraphKey {
  int j;
  const void* arena;
  const void* acc;
  const void* out;
  const void* bases;
  bool overwrite;
  int variant;  // the context's forced GEMM tile variant when captured (-1: the plan's)
  bool operator<(const GraphKey& o) const {
    if (j != o.j) return j < o.j;
    if (variant != o.variant) return variant < o.variant;
    if (overwrite != o.overwrite) return overwrite < o.overwrite;
    if (arena != o.arena) return arena < o.arena;
    if (acc != o.acc) return acc < o.acc;
    if (out != o.out) return out < o.out;
    return bases < o.bases;
  }
};

struct Plan {
  std::shared_ptr<Net> net_ref;       // keeps the network alive (destroyed last)
  Net* net = nullptr;
  std::vector<std::array<int, 2>> pairs;
  std::vector<int> sliced;
  std::vector<int64_t> suffix_prod;   // suffix_prod[j] = slices per chunk with j batched labels
  int64_t n_slices = 1;
  tnc_prec prec = TNC_PREC_C64;
  tnc_cgemm form = TNC_GEMM_4M;
  int64_t max_chunk_user = -1;
  int grouping = 1;                   // level-grouped launches
  int store_order = 0;                // 0: GEMM epilogue stores in consumer order; 1: separate transpose
  std::vector<char> volatile_leaf;    // per leaf: data changes between runs (never cached)
  void* host_res = nullptr;           // pinned staging of tnc_contract's result
  size_t host_res_bytes = 0;
  int graph = 0;
  int profile = 0;
  int j_max = 0;
  std::vector<std::unique_ptr<ChunkPlan>> chunks;   // index j
  std::vector<StepTimer> timers;                    // per step, then preps, reductions
  std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> pending;  // profiling events
  DeviceBuf acc;         // complex128 result accumulator (synchronous calls)
  DeviceBuf norm;        // one double
  std::mutex mu;         // guards lazy chunk building and key_prefix
  std::string key_prefix;  // structure_key's part fixed at creation (built on first use)
  std::mutex graph_mu;   // guards the graph cache
  std::map<GraphKey, hipGraphExec_t> graphs;
  hipStream_t capture_stream = nullptr;
  ~Plan();
  ChunkPlan& chunk(int j);
  // Destroy every captured graph (after the context's stream is drained):
  // the chunk plans or their tile variants changed.
  void drop_graphs();
};

// TNC_E_BUSY while the context serves: plans, networks and launch settings
// that the server's workers read are not changed under them.
void refuse_while_serving(const Ctx& c, const char* what);

// planner.cpp
void validate_net(Net& net);
void validate_path(const Net& net, const std::vector<std::array<int, 2>>& pairs);
std::unique_ptr<ChunkPlan> build_chunk(const Plan& plan, int j);
void choose_chunking(Plan& plan, size_t budget);
size_t run_extra_bytes(const ChunkPlan& cp, int64_t n_chunks);

// distplan.cpp
void plan_distribution(const Plan& plan, int P, double large_bytes, const tnc_dist_hw& hw,
                       std::vector<tnc_dist_step>& out, double& total, double& moved);

// autotune.cpp
int default_variant(tnc_prec prec, tnc_cgemm form, int64_t h, int64_t m, int64_t n);
void load_tune_cache(Ctx& c);
void assign_variants(const Plan& plan, ChunkPlan& cp, bool tune);

// executor.cpp
void materialize(const Net& net, ChunkPlan& cp, hipStream_t stream);
struct RunArgs {
  int64_t first = 0, count = 1;
  char* arena = nullptr;        // workspace (peak + extras)
  size_t arena_bytes = 0;
  double2* acc = nullptr;       // device accumulator (n_result complex128)
  float2* direct_out = nullptr; // single-slice runs: the last step writes here, no reduction
  hipStream_t stream = nullptr;
  bool fresh_acc = false;       // acc holds garbage: the first chunk's reduction overwrites it
};
void run_plan(Plan& plan, const RunArgs& a);
// Arena bytes run_plan needs for a slice range (intermediates of the largest
// chunk, the current chunk's leaf bases, every chunk's leaf bases).
int64_t run_workspace_bytes(Plan& plan, int64_t first, int64_t count);
void drain_profile(Plan& plan);
// Lockstep execution of runs of plans with one structure (fused serving
// jobs): structure_key identifies plans and slice ranges that can run
// together; run_lockstep needs `cap` >= lockstep_table_bytes bytes of pinned
// host memory and of device memory for the job's tables, and every run's
// RunArgs on `stream`.
struct LockstepRun {
  Plan* plan = nullptr;
  RunArgs a;
};
std::string structure_key(Plan& plan, int64_t first, int64_t count);
// What a run contributes to a lockstep job: its bytes of the job's tables,
// the number of sub-tables (each aligned to 256 bytes), and the launches
// the run issues on its own (eager; the measure of how launch-bound it is).
struct LockstepInfo {
  size_t bytes_per_run = 0;
  int64_t parts = 0;
  int64_t launches = 0;
};
LockstepInfo lockstep_info(Plan& plan, int64_t first, int64_t count);
size_t lockstep_table_bytes(const LockstepInfo& t, int n_runs);
void run_lockstep(std::vector<LockstepRun>& runs, void* host_tables, void* dev_tables, size_t cap,
                  hipStream_t stream);
std::vector<std::pair<int, int64_t>> decompose(const Plan& plan, int64_t first, int64_t count);

}  // namespace tnc

// Handles own a reference each: a plan keeps its network alive and a network
// its context, so handles may be destroyed in any order.
// Body of every C entry point: status codes and tnc_last_error() only,
// nothing thrown across the ABI (allocation failures -> TNC_E_NOMEM, other
// standard exceptions -> TNC_E_ARG).
#define TNC_TRY            \
  tnc::g_error_clear();    \
  try {
#define TNC_CATCH                                   \
  }                                                 \
  catch (const tnc::Error& e) {                     \
    tnc::g_error_set(e.msg);                        \
    return e.code;                                  \
  }                                                 \
  catch (const std::bad_alloc&) {                   \
    tnc::g_error_set("host allocation failed");     \
    return TNC_E_NOMEM;                             \
  }                                                 \
  catch (const std::exception& e) {                 \
    tnc::g_error_set(e.what());                     \
    return TNC_E_ARG;                               \
  }                                                 \
  return TNC_OK;

struct tnc_ctx_s {
  std::shared_ptr<tnc::Ctx> c;
};
struct tnc_net_s {
  std::shared_ptr<tnc::Net> n;
};
struct tnc_plan_s {
  std::shared_ptr<tnc::Plan> p;
};
namespace tnc {
struct Batcher;
}
struct tnc_batcher_s {
  std::shared_ptr<tnc::Batcher> b;
};
