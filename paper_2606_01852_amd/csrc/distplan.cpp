// Communication-aware mode-distribution planning (paper Sec. IV-B), on the
// host.  The plan is not executed on several GPUs here; this is the offline
// planner that would drive such an execution.
//
//  * a step is large when its operands or output reach `large_bytes`;
//  * a use-chain starts at a large step and follows the tensor's consumers
//    (its descendants) up the tree, ending at the last large step on the way;
//  * the first equation distributes its output on the shortest prefix of its
//    mode order whose extents multiply to >= P (Eq. (4)); modes are tracked
//    by label, so the tag each label carries (the step that sums it) decides
//    which equation sums a distributed mode;
//  * every later equation keeps the inherited modes or redistributes to a
//    fresh prefix; a distributed mode summed by the next equation forces the
//    redistribution; the chain ends with a gather;
//  * costs: Eq. (5)-(7) with per-device bytes and FLOPs; a DP over the set of
//    distributed modes picks the cheapest schedule, backtracing the
//    redistribution points.
#include <algorithm>
#include <cmath>
#include <map>

#include "core.hpp"

namespace tnc {

namespace {

struct Eq {
  int step = -1;
  std::vector<int> order;       // output modes
  double a = 0, b = 0, c = 0;   // elements: chain operand, other operand, output
  double ops = 0;               // complex multiply-adds
  std::vector<int> next_summed; // output labels summed by the next equation
};

using Modes = std::vector<int>;

Modes prefix_modes(const Eq& e, const std::vector<int64_t>& ext, int P) {
  Modes out;
  int64_t prod = 1;
  for (int l : e.order) {
    if (prod >= P) break;
    out.push_back(l);
    prod *= ext[l];
  }
  if (prod < P) out.clear();
  return out;
}

bool meets(const Modes& d, const std::vector<int>& labels) {
  for (int l : d)
    if (std::find(labels.begin(), labels.end(), l) != labels.end()) return true;
  return false;
}

double t_gemm(const Eq& e, int P, const tnc_dist_hw& hw) {
  const double d_rw = 8.0 * (e.a / P + e.b + e.c / P);
  const double flops = 8.0 * e.ops / P;
  return std::max(d_rw / hw.hbm_bytes_per_s, flops / hw.flops_per_s);
}

double t_comm(const Eq& e, const std::vector<int64_t>& ext, int P, const tnc_dist_hw& hw, const Modes& old_d,
              const Modes& new_d) {
  int last = -1;
  for (size_t q = 0; q < e.order.size(); ++q) {
    const int l = e.order[q];
    if (std::find(old_d.begin(), old_d.end(), l) != old_d.end() ||
        std::find(new_d.begin(), new_d.end(), l) != new_d.end())
      last = static_cast<int>(q);
  }
  double inner = 1;
  for (size_t q = last + 1; q < e.order.size(); ++q) inner *= static_cast<double>(ext[e.order[q]]);
  const double s_blk = 8.0 * inner;
  const double n_blk = std::ceil(8.0 * e.c / P / s_blk);
  return 8.0 * e.c * (P - 1) / (P * hw.net_bytes_per_s) + n_blk * std::max(hw.latency_s, s_blk / hw.net_bytes_per_s);
}

double t_gather(const Eq& e, int P, const tnc_dist_hw& hw) {
  return 8.0 * e.c * (P - 1) / (P * hw.net_bytes_per_s);
}

}  // namespace

void plan_distribution(const Plan& plan, int P, double large_bytes, const tnc_dist_hw& hw,
                       std::vector<tnc_dist_step>& out, double& total, double& moved) {
  const ChunkPlan& cp = *plan.chunks[0];
  const Net& net = *plan.net;
  const std::vector<int64_t>& ext = net.extents;
  const int n = net.n_tensors;
  const int ns = static_cast<int>(cp.steps.size());
  std::vector<int> consumer(n + ns, -1);
  for (int s = 0; s < ns; ++s) {
    consumer[plan.pairs[s][0]] = s;
    consumer[plan.pairs[s][1]] = s;
  }
  auto bytes = [&](int id) { return 8.0 * static_cast<double>(cp.numel[id]); };
  auto large = [&](int s) {
    const StepPlan& sp = cp.steps[s];
    return std::max({bytes(sp.A), bytes(sp.B), bytes(sp.C)}) >= large_bytes;
  };
  std::vector<char> covered(ns, 0);
  total = 0;
  moved = 0;
  int chain_id = 0;
  for (int s0 = 0; s0 < ns; ++s0) {
    if (covered[s0] || !large(s0)) continue;
    std::vector<int> chain;
    for (int t = s0; t >= 0 && !covered[t]; t = consumer[cp.steps[t].C]) chain.push_back(t);
    while (!chain.empty() && !large(chain.back())) chain.pop_back();
    for (int t : chain) covered[t] = 1;
    // equations of the chain
    std::vector<Eq> eqs(chain.size());
    for (size_t i = 0; i < chain.size(); ++i) {
      const StepPlan& sp = cp.steps[chain[i]];
      Eq& e = eqs[i];
      e.step = chain[i];
      e.order = cp.order[sp.C];
      int main_id;
      if (i == 0)
        main_id = bytes(sp.A) >= bytes(sp.B) ? sp.A : sp.B;
      else
        main_id = cp.steps[chain[i - 1]].C;
      const int other = main_id == sp.A ? sp.B : sp.A;
      e.a = static_cast<double>(cp.numel[main_id]);
      e.b = static_cast<double>(cp.numel[other]);
      e.c = static_cast<double>(cp.numel[sp.C]);
      e.ops = static_cast<double>(sp.h) * sp.m * sp.n * sp.k;
      if (i + 1 < chain.size()) {
        for (int l : cp.steps[chain[i + 1]].K)
          if (std::find(e.order.begin(), e.order.end(), l) != e.order.end()) e.next_summed.push_back(l);
      }
    }
    // DP over the distributed modes of each equation's output
    struct Cell {
      double cost;
      Modes prev;
      bool redist;
    };
    std::vector<std::map<Modes, Cell>> dp(eqs.size());
    const Modes d0 = prefix_modes(eqs[0], ext, P);
    if (d0.empty() || meets(d0, eqs[0].next_summed)) continue;  // cannot be split P ways
    dp[0][d0] = {t_gemm(eqs[0], P, hw), {}, false};
    for (size_t i = 1; i < eqs.size(); ++i) {
      const double tg = t_gemm(eqs[i], P, hw);
      const Modes fresh = prefix_modes(eqs[i], ext, P);
      for (const auto& kv : dp[i - 1]) {
        const Modes& d = kv.first;
        const double base = kv.second.cost + tg;
        auto relax = [&](const Modes& nd, double c, bool r) {
          auto it = dp[i].find(nd);
          if (it == dp[i].end() || c < it->second.cost) dp[i][nd] = {c, d, r};
        };
        if (!meets(d, eqs[i].next_summed)) relax(d, base, false);  // keep
        if (!fresh.empty() && !meets(fresh, eqs[i].next_summed))
          relax(fresh, base + t_comm(eqs[i], ext, P, hw, d, fresh), true);  // redistribute
      }
    }
    if (dp.back().empty()) continue;
    auto best = dp.back().begin();
    double best_cost = 1e300;
    for (auto it = dp.back().begin(); it != dp.back().end(); ++it) {
      const double c = it->second.cost + t_gather(eqs.back(), P, hw);
      if (c < best_cost) {
        best_cost = c;
        best = it;
      }
    }
    total += best_cost;
    // backtrace
    std::vector<Modes> ds(eqs.size());
    std::vector<bool> rs(eqs.size(), false);
    Modes cur = best->first;
    for (int i = static_cast<int>(eqs.size()) - 1; i >= 0; --i) {
      ds[i] = cur;
      const Cell& cell = dp[i].at(cur);
      rs[i] = cell.redist;
      cur = cell.prev;
    }
    for (size_t i = 0; i < eqs.size(); ++i) {
      tnc_dist_step r{};
      r.chain = chain_id;
      r.step = eqs[i].step;
      r.state = i == 0 ? 0 : (rs[i] ? 2 : 1);
      r.n_dist = static_cast<int32_t>(std::min<size_t>(ds[i].size(), 16));
      for (int q = 0; q < r.n_dist; ++q) r.dist[q] = ds[i][q];
      r.t_gemm_s = t_gemm(eqs[i], P, hw);
      r.t_comm_s = rs[i] ? t_comm(eqs[i], ext, P, hw, ds[i - 1], ds[i]) : 0.0;
      r.out_bytes = 8.0 * eqs[i].c;
      if (rs[i]) moved += 8.0 * eqs[i].c * (P - 1) / P;
      out.push_back(r);
    }
    ++chain_id;
  }
}

}  // namespace tnc
