// Host-side driver of the C ABI for the sanitizer tests (AddressSanitizer,
// UndefinedBehaviorSanitizer or ThreadSanitizer on the host code; no GPU is
// touched: every call goes to a host-only context).
//
// Input (whitespace-separated integers, one network per file):
//   n_tensors  then per tensor: rank, labels...
//   n_labels   then the extent of every label
//   n_open     then the open labels
//   n_steps    then the SSA pairs
//   n_sliced   then the sliced labels
//   batch_label (-1: none), then n_leaves and the leaves of a batcher
// For each network the driver plans it (both execution orders and store orders, every chunk
// size), queries every step and order, plans its distribution over 2, 4 and
// 8 devices, creates and destroys a batcher when asked, and checks that
// malformed paths come back as status codes; a fixed set of malformed
// networks, paths, slices and kernel arguments runs first.  Prints
// "ok <file>" per file.  With --threads N first, N threads each plan every
// network on a context of their own at the same time (for ThreadSanitizer:
// contexts share no mutable state).  Both modes end with a serving run on a
// host-only context ("ok serving"): its server admits and queues requests
// and batcher rows from several submitting threads with its own worker
// threads, and completes each without executing it.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <thread>
#include <vector>

#include "../include/tnc.h"

namespace {

std::atomic<int> fails{0};

void expect(bool cond, const char* what, const char* file) {
  if (!cond) {
    std::fprintf(stderr, "FAIL %s: %s (%s)\n", file, what, tnc_last_error());
    ++fails;
  }
}

struct NetFile {
  int n_tensors = 0;
  std::vector<int32_t> ranks, labels;
  std::vector<int64_t> extents;
  std::vector<int32_t> open, pairs, sliced, batch_leaves;
  int batch_label = -1;
};

bool read_net(const char* path, NetFile& f) {
  std::ifstream in(path);
  if (!in) return false;
  in >> f.n_tensors;
  for (int t = 0; t < f.n_tensors; ++t) {
    int r = 0;
    in >> r;
    f.ranks.push_back(r);
    for (int q = 0; q < r; ++q) {
      int l = 0;
      in >> l;
      f.labels.push_back(l);
    }
  }
  int n = 0;
  in >> n;
  f.extents.resize(n);
  for (auto& e : f.extents) in >> e;
  in >> n;
  f.open.resize(n);
  for (auto& o : f.open) in >> o;
  in >> n;
  f.pairs.resize(2 * n);
  for (auto& p : f.pairs) in >> p;
  in >> n;
  f.sliced.resize(n);
  for (auto& s : f.sliced) in >> s;
  in >> f.batch_label >> n;
  f.batch_leaves.resize(n);
  for (auto& b : f.batch_leaves) in >> b;
  return static_cast<bool>(in);
}

void exercise(tnc_ctx ctx, const NetFile& f, const char* file) {
  tnc_net net = nullptr;
  expect(tnc_net_create(ctx, f.n_tensors, f.ranks.data(), f.labels.data(), static_cast<int32_t>(f.extents.size()),
                        f.extents.data(), static_cast<int32_t>(f.open.size()), f.open.data(), nullptr, TNC_IN_C64,
                        &net) == TNC_OK,
         "net_create", file);
  if (!net) return;
  const int32_t n_steps = static_cast<int32_t>(f.pairs.size() / 2);
  tnc_plan plan = nullptr;
  expect(tnc_plan_create(net, n_steps, f.pairs.data(), static_cast<int32_t>(f.sliced.size()), f.sliced.data(),
                         TNC_PREC_C64, TNC_GEMM_4M, &plan) == TNC_OK,
         "plan_create", file);
  if (plan) {
    tnc_plan_info info;
    for (int mode = 0; mode < 4; ++mode) {
      const int grouping = mode & 1 ? 0 : 1, store = mode >> 1;
      expect(tnc_plan_set_grouping(plan, grouping) == TNC_OK, "set_grouping", file);
      expect(tnc_plan_set_store_order(plan, store) == TNC_OK, "set_store_order", file);
      for (int64_t cap : {int64_t{1}, int64_t{4}, int64_t{-1}}) {
        expect(tnc_plan_set_max_chunk(plan, cap) == TNC_OK, "set_max_chunk", file);
        expect(tnc_plan_get_info(plan, &info) == TNC_OK, "get_info", file);
        for (int32_t s = 0; s < n_steps; ++s) {
          tnc_step_info st;
          expect(tnc_plan_get_step(plan, s, &st) == TNC_OK, "get_step", file);
          expect(tnc_plan_get_batch_step(plan, s, &st) == TNC_OK, "get_batch_step", file);
        }
      }
    }
    expect(tnc_plan_set_store_order(plan, 2) == TNC_E_ARG, "store order out of range", file);
    std::vector<int32_t> order(64);
    for (int32_t id = 0; id < f.n_tensors + n_steps; ++id) {
      int32_t rank = 0;
      expect(tnc_plan_get_order(plan, id, order.data(), 64, &rank) == TNC_OK, "get_order", file);
    }
    tnc_step_info st;
    expect(tnc_plan_get_step(plan, n_steps, &st) == TNC_E_ARG, "step out of range", file);
    tnc_dist_hw hw{5.3e12, 1.4e14, 1.0e11, 2e-6};
    std::vector<tnc_dist_step> steps(4096);
    for (int P : {2, 4, 8}) {
      int32_t n_out = 0;
      double total = 0, moved = 0;
      expect(tnc_plan_distribute(plan, P, 1e3, &hw, steps.data(), static_cast<int32_t>(steps.size()), &n_out,
                                 &total, &moved) == TNC_OK,
             "distribute", file);
    }
    if (f.batch_label >= 0) {
      tnc_batcher b = nullptr;
      expect(tnc_batcher_create(plan, f.batch_label, static_cast<int32_t>(f.batch_leaves.size()),
                                f.batch_leaves.data(), &b) == TNC_OK,
             "batcher_create", file);
      tnc_batcher b2 = nullptr;
      expect(tnc_batcher_create(plan, f.batch_label, static_cast<int32_t>(f.batch_leaves.size()),
                                f.batch_leaves.data(), &b2) == TNC_E_BUSY,
             "second batcher refused", file);
      expect(tnc_batcher_destroy(b) == TNC_OK, "batcher_destroy", file);
    }
    expect(tnc_plan_destroy(plan) == TNC_OK, "plan_destroy", file);
  }
  // malformed paths: a repeated id, an id out of range
  if (n_steps > 0) {
    std::vector<int32_t> bad = f.pairs;
    bad[1] = bad[0];
    tnc_plan p2 = nullptr;
    expect(tnc_plan_create(net, n_steps, bad.data(), 0, nullptr, TNC_PREC_C64, TNC_GEMM_4M, &p2) != TNC_OK,
           "repeated id rejected", file);
    bad = f.pairs;
    bad[0] = f.n_tensors + n_steps + 7;
    expect(tnc_plan_create(net, n_steps, bad.data(), 0, nullptr, TNC_PREC_C64, TNC_GEMM_4M, &p2) != TNC_OK,
           "id out of range rejected", file);
  }
  expect(tnc_net_destroy(net) == TNC_OK, "net_destroy", file);
}

tnc_status make_net(tnc_ctx ctx, const std::vector<int32_t>& ranks, const std::vector<int32_t>& labels,
                    const std::vector<int64_t>& ext, const std::vector<int32_t>& open, tnc_net* out) {
  *out = nullptr;
  return tnc_net_create(ctx, static_cast<int32_t>(ranks.size()), ranks.data(), labels.data(),
                        static_cast<int32_t>(ext.size()), ext.data(), static_cast<int32_t>(open.size()),
                        open.empty() ? nullptr : open.data(), nullptr, TNC_IN_C64, out);
}

// Arguments every entry point must turn into a status code, never a crash.
void malformed(tnc_ctx ctx) {
  const char* F = "malformed";
  tnc_net net = nullptr;
  // networks: label out of range, label repeated in a tensor, extent 0, an
  // open label repeated or on no tensor, a negative rank, no tensors, a label
  // held by three tensors, an intermediate past int64
  expect(make_net(ctx, {2, 1}, {0, 3, 0}, {2, 2}, {}, &net) == TNC_E_ARG, "label out of range", F);
  expect(make_net(ctx, {2, 1}, {0, 0, 0}, {2}, {}, &net) == TNC_E_ARG, "label repeated", F);
  expect(make_net(ctx, {1, 1}, {0, 0}, {0}, {}, &net) == TNC_E_ARG, "extent 0", F);
  expect(make_net(ctx, {1, 1}, {0, 1}, {2, 2}, {0, 0}, &net) == TNC_E_ARG, "open repeated", F);
  expect(make_net(ctx, {1, 1}, {0, 0}, {2, 2}, {1}, &net) == TNC_E_ARG, "open on no tensor", F);
  expect(make_net(ctx, {-1, 1}, {0, 0}, {2}, {}, &net) == TNC_E_ARG, "negative rank", F);
  expect(tnc_net_create(ctx, 0, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, TNC_IN_C64, &net) == TNC_E_ARG,
         "no tensors", F);
  expect(make_net(ctx, {1, 1, 1}, {0, 0, 0}, {2}, {}, &net) == TNC_E_ARG, "hyperedge", F);
  {
    const int32_t r[2] = {1, 1}, l[2] = {0, 0};
    const int64_t e[1] = {2};
    expect(tnc_net_create(ctx, 2, r, l, 1, e, 0, nullptr, nullptr, 5, &net) == TNC_E_ARG, "input type", F);
  }
  expect(tnc_net_create(nullptr, 1, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, TNC_IN_C64, &net) == TNC_E_ARG,
         "null ctx", F);
  {
    // A(a b c d) B(c d e f): the product's open labels a b e f at 2^20 each
    const std::vector<int64_t> big = {1 << 20, 1 << 20, 2, 2, 1 << 20, 1 << 20};
    if (make_net(ctx, {4, 4}, {0, 1, 2, 3, 2, 3, 4, 5}, big, {0, 1, 4, 5}, &net) == TNC_OK) {
      const int32_t pair[2] = {0, 1};
      tnc_plan p = nullptr;
      expect(tnc_plan_create(net, 1, pair, 0, nullptr, TNC_PREC_C64, TNC_GEMM_4M, &p) != TNC_OK, "size overflow", F);
      tnc_net_destroy(net);
    } else {
      expect(false, "overflowing net refused at creation", F);
    }
  }
  // plans over A(0 1) B(1 2) C(2 0), closed: wrong step counts, bad slices,
  // bad enums, the split precision in the 3M form
  expect(make_net(ctx, {2, 2, 2}, {0, 1, 1, 2, 2, 0}, {3, 4, 5}, {}, &net) == TNC_OK, "triangle", F);
  if (net) {
    tnc_plan p = nullptr;
    const int32_t good[4] = {0, 1, 3, 2};
    const int32_t self[4] = {0, 0, 3, 2};
    const int32_t fwd[4] = {0, 4, 3, 2};
    expect(tnc_plan_create(net, 1, good, 0, nullptr, TNC_PREC_C64, TNC_GEMM_4M, &p) == TNC_E_PATH, "short path", F);
    expect(tnc_plan_create(net, 2, self, 0, nullptr, TNC_PREC_C64, TNC_GEMM_4M, &p) == TNC_E_PATH, "self pair", F);
    expect(tnc_plan_create(net, 2, fwd, 0, nullptr, TNC_PREC_C64, TNC_GEMM_4M, &p) == TNC_E_PATH, "forward id", F);
    expect(tnc_plan_create(net, 2, nullptr, 0, nullptr, TNC_PREC_C64, TNC_GEMM_4M, &p) == TNC_E_ARG, "null path", F);
    const int32_t sl_bad[2] = {7, 0}, sl_rep[2] = {1, 1};
    expect(tnc_plan_create(net, 2, good, 1, sl_bad, TNC_PREC_C64, TNC_GEMM_4M, &p) == TNC_E_ARG, "slice range", F);
    expect(tnc_plan_create(net, 2, good, 2, sl_rep, TNC_PREC_C64, TNC_GEMM_4M, &p) == TNC_E_ARG, "slice twice", F);
    expect(tnc_plan_create(net, 2, good, 0, nullptr, 9, TNC_GEMM_4M, &p) == TNC_E_ARG,
           "unknown precision", F);
    expect(tnc_plan_create(net, 2, good, 0, nullptr, TNC_PREC_C64, 9, &p) == TNC_E_ARG,
           "unknown form", F);
    expect(tnc_plan_create(net, 2, good, 0, nullptr, TNC_PREC_BF16X3, -1, &p) == TNC_E_ARG, "negative form", F);
    p = nullptr;
    expect(tnc_plan_create(net, 2, good, 0, nullptr, TNC_PREC_BF16X3, TNC_GEMM_3M, &p) == TNC_OK, "split 3M", F);
    if (p) expect(tnc_plan_destroy(p) == TNC_OK, "split 3M destroy", F);
    p = nullptr;
    const int32_t sl[1] = {1};
    expect(tnc_plan_create(net, 2, good, 1, sl, TNC_PREC_C64, TNC_GEMM_4M, &p) == TNC_OK, "triangle plan", F);
    if (p) {
      tnc_dist_hw hw{5.3e12, 1.4e14, 1.0e11, 2e-6};
      int32_t n_out = 0;
      double total = 0, moved = 0;
      tnc_dist_step steps[8];
      expect(tnc_plan_distribute(p, 1, 1e3, &hw, steps, 8, &n_out, &total, &moved) == TNC_E_ARG, "one gpu", F);
      tnc_dist_hw neg{-1.0, 1.4e14, 1.0e11, 2e-6};
      expect(tnc_plan_distribute(p, 4, 1e3, &neg, steps, 8, &n_out, &total, &moved) == TNC_E_ARG, "bad hw", F);
      // cap 0 still reports the step count (0 here: extents 3 and 5 do not
      // split four ways); a short cap writes only its part
      expect(tnc_plan_distribute(p, 4, 1.0, &hw, nullptr, 0, &n_out, &total, &moved) == TNC_OK && n_out >= 0,
             "distribute cap 0", F);
      const int32_t full = n_out;
      expect(tnc_plan_distribute(p, 4, 1.0, &hw, steps, 1, &n_out, &total, &moved) == TNC_OK && n_out == full,
             "distribute cap 1", F);
      int32_t order[1], rank = 0;
      expect(tnc_plan_get_order(p, 3, order, 1, &rank) == TNC_OK, "order cap short", F);
      expect(tnc_plan_get_order(p, 5, order, 1, &rank) == TNC_E_ARG, "order id", F);
      expect(tnc_plan_get_order(p, -1, order, 1, &rank) == TNC_E_ARG, "order id negative", F);
      tnc_step_info st;
      expect(tnc_plan_get_step(p, -1, &st) == TNC_E_ARG, "negative step", F);
      double out[2];
      expect(tnc_contract(p, 0, 1, out) == TNC_E_UNSUPPORTED, "host-only contract", F);
      const int32_t leaf[1] = {0};
      tnc_batcher b = nullptr;
      expect(tnc_batcher_create(p, 0, 1, leaf, &b) == TNC_E_ARG, "batch label closed", F);
      expect(tnc_batcher_create(p, 0, 0, leaf, &b) == TNC_E_ARG, "batcher with no leaves", F);
      tnc_plan_destroy(p);
    }
    tnc_net_destroy(net);
  }
  // permutes: checked before any device work, then refused on a host context
  {
    const int64_t ext[3] = {4, 5, 6}, huge[3] = {int64_t{1} << 30, int64_t{1} << 30, 64};
    const int32_t perm[3] = {2, 0, 1}, dup[3] = {2, 2, 1}, out_of[3] = {3, 0, 1};
    float dummy[2];
    expect(tnc_permute(ctx, dummy, dummy, 3, ext, dup) == TNC_E_ARG, "perm repeated", F);
    expect(tnc_permute(ctx, dummy, dummy, 3, ext, out_of) == TNC_E_ARG, "perm out of range", F);
    expect(tnc_permute(ctx, dummy, dummy, 3, huge, perm) == TNC_E_ARG, "permute size overflow", F);
    expect(tnc_permute(ctx, dummy, dummy, 3, ext, perm) == TNC_E_UNSUPPORTED, "permute on host", F);
    expect(tnc_batched_cgemm(ctx, 1, 0, 4, 4, dummy, 0, dummy, 0, dummy, TNC_PREC_C64, TNC_GEMM_4M) == TNC_E_ARG,
           "gemm m 0", F);
    expect(tnc_batched_cgemm(ctx, 1, 4, 4, 4, dummy, 0, dummy, 0, dummy, 7, TNC_GEMM_4M) == TNC_E_ARG,
           "gemm precision", F);
    expect(tnc_batched_cgemm(ctx, 1, 4, 4, 4, dummy, 0, dummy, 0, dummy, TNC_PREC_C64, -3) == TNC_E_ARG,
           "gemm form", F);
    tnc_ctx sized = nullptr;
    expect(tnc_ctx_create(-1, nullptr, 0, nullptr, &sized) == TNC_OK, "host context without arena", F);
    expect(tnc_serve_start(sized, 4, 16) == TNC_E_ARG, "serve without an arena size", F);
    tnc_ctx_destroy(sized);
    expect(tnc_serve_start(ctx, 0, 16) == TNC_E_ARG, "serve with no slots", F);
  }
  expect(tnc_plan_destroy(nullptr) == TNC_OK, "destroy null plan", F);
  expect(tnc_net_destroy(nullptr) == TNC_OK, "destroy null net", F);
}

int64_t numel_of(const NetFile& f, int t) {
  int64_t pos = 0;
  for (int u = 0; u < t; ++u) pos += f.ranks[u];
  int64_t n = 1;
  for (int q = 0; q < f.ranks[t]; ++q) n *= f.extents[f.labels[pos + q]];
  return n;
}

// Serving on a host-only context: `submitters` threads submit whole-plan
// requests and batcher rows, poll and wait, while the server's worker
// threads admit them by planned arena bytes; every request must complete
// with TNC_E_UNSUPPORTED.  Calls that would change a plan or a network
// under the workers must be refused while it serves.  Two rounds: the
// second with the heavy lane on and a batcher destroyed while its rows may
// still be queued.
void serve_exercise(const std::vector<NetFile>& files, int submitters) {
  const char* F = "serving";
  tnc_ctx ctx = nullptr;
  if (tnc_ctx_create(-1, nullptr, size_t{64} << 30, nullptr, &ctx) != TNC_OK) {
    expect(false, "host context", F);
    return;
  }
  struct Entry {
    tnc_net net = nullptr;
    tnc_plan plan = nullptr;
    tnc_batcher batcher = nullptr;
    int64_t n_result = 1, n_slices = 1, row_result = 1;
    std::vector<std::vector<double>> rows;  // per listed leaf: one row of complex128 values
  };
  std::vector<Entry> es;
  for (const NetFile& f : files) {
    Entry e;
    if (tnc_net_create(ctx, f.n_tensors, f.ranks.data(), f.labels.data(), static_cast<int32_t>(f.extents.size()),
                       f.extents.data(), static_cast<int32_t>(f.open.size()), f.open.data(), nullptr, TNC_IN_C64,
                       &e.net) != TNC_OK)
      continue;
    const int32_t n_steps = static_cast<int32_t>(f.pairs.size() / 2);
    if (tnc_plan_create(e.net, n_steps, f.pairs.data(), static_cast<int32_t>(f.sliced.size()), f.sliced.data(),
                        TNC_PREC_C64, TNC_GEMM_4M, &e.plan) != TNC_OK) {
      tnc_net_destroy(e.net);
      continue;  // too large for the arena
    }
    tnc_plan_info info;
    expect(tnc_plan_get_info(e.plan, &info) == TNC_OK, "serving info", F);
    e.n_result = info.n_result;
    e.n_slices = info.n_slices;
    if (e.n_result > (1 << 16)) {  // host outputs of every request stay small
      tnc_plan_destroy(e.plan);
      tnc_net_destroy(e.net);
      continue;
    }
    if (f.batch_label >= 0) {
      expect(tnc_batcher_create(e.plan, f.batch_label, static_cast<int32_t>(f.batch_leaves.size()),
                                f.batch_leaves.data(), &e.batcher) == TNC_OK,
             "serving batcher", F);
      const int64_t B = f.extents[f.batch_label];
      e.row_result = e.n_result / B;
      for (int t : f.batch_leaves) e.rows.emplace_back(static_cast<size_t>(2 * numel_of(f, t) / B), 0.5);
    }
    es.push_back(std::move(e));
  }
  expect(!es.empty(), "networks to serve", F);
  for (int round = 0; round < 2 && !es.empty(); ++round) {
    expect(tnc_serve_start(ctx, 6, 1 << 14) == TNC_OK, "serve_start", F);
    expect(tnc_serve_start(ctx, 6, 16) == TNC_E_BUSY, "second server", F);
    expect(tnc_serve_set_heavy(ctx, round ? 1e6 : 0.0, 2) == TNC_OK, "heavy lane", F);
    expect(tnc_serve_set_fusion(ctx, round ? 4 : 1, round ? 1e300 : 134217728.0) == TNC_OK, "fusion", F);
    expect(tnc_serve_set_fusion(ctx, 0, 1.0) == TNC_E_ARG, "fusion limit", F);
    expect(tnc_serve_set_fusion(ctx, 4, 0.0) == TNC_E_ARG, "fusion criterion", F);
    tnc_plan p0 = es[0].plan;
    int32_t rank = 0;
    double out[2] = {0, 0};
    expect(tnc_plan_set_max_chunk(p0, 4) == TNC_E_BUSY, "set_max_chunk while serving", F);
    expect(tnc_plan_set_graph(p0, 1) == TNC_E_BUSY, "set_graph while serving", F);
    expect(tnc_plan_set_grouping(p0, 0) == TNC_E_BUSY, "set_grouping while serving", F);
    expect(tnc_plan_set_profile(p0, 1) == TNC_E_BUSY, "set_profile while serving", F);
    expect(tnc_plan_autotune(p0) == TNC_E_BUSY, "autotune while serving", F);
    expect(tnc_ctx_set_gemm_variant(ctx, 1) == TNC_E_BUSY, "forced variant while serving", F);
    expect(tnc_contract(p0, 0, 1, out) == TNC_E_BUSY, "contract while serving", F);
    expect(tnc_contract_async(p0, 0, 1, out, TNC_OUT_C128) == TNC_E_BUSY, "contract_async while serving", F);
    expect(tnc_net_set_tensor(es[0].net, 0, out, TNC_IN_C128) == TNC_E_BUSY, "set_tensor while serving", F);
    expect(tnc_net_set_tensor_device(es[0].net, 0, out) == TNC_E_BUSY, "set_tensor_device while serving", F);
    expect(tnc_plan_get_order(p0, 0, nullptr, 0, &rank) == TNC_OK, "queries stay allowed", F);
    std::vector<std::thread> pool;
    for (int t = 0; t < submitters; ++t)
      pool.emplace_back([&, t] {
        std::vector<std::pair<tnc_req, std::vector<double>>> mine;
        for (int i = 0; i < 48; ++i) {
          const Entry& e = es[(t + i) % es.size()];
          std::vector<double> res;
          tnc_req id = 0;
          tnc_status st;
          if (!e.rows.empty()) {
            res.assign(static_cast<size_t>(2 * e.row_result), 0.0);
            std::vector<const void*> ptrs;
            for (const auto& r : e.rows) ptrs.push_back(r.data());
            st = tnc_submit_row(ctx, e.batcher, ptrs.data(), TNC_IN_C128, res.data(), &id);
          } else {
            res.assign(static_cast<size_t>(2 * e.n_result), 0.0);
            const int64_t first = i % e.n_slices;
            st = tnc_submit(ctx, e.plan, first, 1 + (e.n_slices - first - 1) * (i % 2), res.data(), &id);
          }
          expect(st == TNC_OK, "submit", F);
          if (st != TNC_OK) continue;
          if (i % 3 == 0) {
            int32_t d = 0;
            double lat = 0;
            const tnc_status ps = tnc_poll(ctx, id, &d, &lat);
            expect(ps == TNC_OK || (d == 1 && ps == TNC_E_UNSUPPORTED), "poll", F);
          }
          mine.emplace_back(id, std::move(res));
        }
        for (auto& m : mine) {
          double lat = -1;
          expect(tnc_wait(ctx, m.first, &lat) == TNC_E_UNSUPPORTED && lat >= 0, "request completes unexecuted", F);
          for (double v : m.second) expect(v == 0.0, "output untouched", F);
        }
        int32_t d = 0;
        if (!mine.empty()) expect(tnc_poll(ctx, mine[0].first, &d, nullptr) == TNC_E_ARG, "collected id unknown", F);
      });
    for (auto& th : pool) th.join();
    if (round == 1)
      for (Entry& e : es)
        if (e.batcher) {
          // rows queued now keep the batcher alive until they are done
          std::vector<const void*> ptrs;
          for (const auto& r : e.rows) ptrs.push_back(r.data());
          std::vector<std::vector<double>> res(8, std::vector<double>(static_cast<size_t>(2 * e.row_result), 0.0));
          std::vector<tnc_req> ids(8, 0);
          for (int i = 0; i < 8; ++i)
            expect(tnc_submit_row(ctx, e.batcher, ptrs.data(), TNC_IN_C128, res[i].data(), &ids[i]) == TNC_OK,
                   "late row", F);
          expect(tnc_batcher_destroy(e.batcher) == TNC_OK, "batcher destroyed while serving", F);
          e.batcher = nullptr;
          for (tnc_req id : ids) expect(tnc_wait(ctx, id, nullptr) == TNC_E_UNSUPPORTED, "late row completes", F);
        }
    int64_t jobs = 0, fused_jobs = 0, fused_requests = 0;
    expect(tnc_serve_get_stats(ctx, &jobs, &fused_jobs, &fused_requests) == TNC_OK && jobs > 0 &&
               fused_requests >= 2 * fused_jobs,
           "serving counters", F);
    expect(tnc_serve_stop(ctx) == TNC_OK, "serve_stop", F);
    expect(tnc_plan_set_max_chunk(p0, -1) == TNC_OK, "set_max_chunk after serving", F);
  }
  for (Entry& e : es) {
    if (e.batcher) tnc_batcher_destroy(e.batcher);
    tnc_plan_destroy(e.plan);
    tnc_net_destroy(e.net);
  }
  tnc_ctx_destroy(ctx);
}

}  // namespace

int threaded(int n_threads, int n_files, char** files) {
  std::vector<NetFile> nets(n_files);
  for (int i = 0; i < n_files; ++i)
    if (!read_net(files[i], nets[i])) {
      std::fprintf(stderr, "cannot read %s\n", files[i]);
      return 2;
    }
  std::vector<std::thread> pool;
  for (int t = 0; t < n_threads; ++t)
    pool.emplace_back([&, t] {
      tnc_ctx ctx = nullptr;
      if (tnc_ctx_create(-1, nullptr, size_t{64} << 30, nullptr, &ctx) != TNC_OK) {
        ++fails;
        return;
      }
      for (int i = 0; i < n_files; ++i) {
        const int f = (i + t) % n_files;  // threads start on different networks
        exercise(ctx, nets[f], files[f]);
        std::printf("ok %s\n", files[f]);
      }
      tnc_ctx_destroy(ctx);
    });
  for (auto& th : pool) th.join();
  serve_exercise(nets, n_threads);
  std::printf("ok serving\n");
  return fails ? 1 : 0;
}

int main(int argc, char** argv) {
  if (argc > 2 && std::strcmp(argv[1], "--threads") == 0) return threaded(std::atoi(argv[2]), argc - 3, argv + 3);
  tnc_ctx ctx = nullptr;
  if (tnc_ctx_create(-1, nullptr, size_t{64} << 30, nullptr, &ctx) != TNC_OK) {
    std::fprintf(stderr, "host context: %s\n", tnc_last_error());
    return 2;
  }
  malformed(ctx);
  std::printf("ok malformed\n");
  std::vector<NetFile> nets;
  for (int i = 1; i < argc; ++i) {
    NetFile f;
    if (!read_net(argv[i], f)) {
      std::fprintf(stderr, "cannot read %s\n", argv[i]);
      return 2;
    }
    exercise(ctx, f, argv[i]);
    std::printf("ok %s\n", argv[i]);
    nets.push_back(std::move(f));
  }
  tnc_ctx_destroy(ctx);
  serve_exercise(nets, 4);
  std::printf("ok serving\n");
  return fails ? 1 : 0;
}
