// Host planner: network and path validation (labels join two tensors, or
// one tensor and the open list: Sec. II-A), the per-step GEMM groups H/M/N/K
// and their costs (Sec. II-B, Eq. (1)-(3)), GEMM-oriented mode reordering
// (Sec. IV-A), slicing as batch labels (Sec. II-C), permutation tables and
// the arena memory plan.  Everything here runs on the host before any
// device work.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "core.hpp"

namespace tnc {

namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t checked_mul(int64_t a, int64_t b) {
  if (a != 0 && b > INT64_MAX / 4 / a) fail(TNC_E_ARG, "tensor size overflows int64");
  return a * b;
}

std::vector<int64_t> row_major(const std::vector<int64_t>& ext) {
  std::vector<int64_t> st(ext.size());
  int64_t s = 1;
  for (int i = static_cast<int>(ext.size()) - 1; i >= 0; --i) {
    st[i] = s;
    s *= ext[i];
  }
  return st;
}

}  // namespace

// ------------------------------------------------------------------ validation
void validate_net(Net& net) {
  const int L = static_cast<int>(net.extents.size());
  for (int l = 0; l < L; ++l)
    if (net.extents[l] < 1) fail(TNC_E_ARG, "extent of label " + std::to_string(l) + " < 1");
  std::vector<int> cnt(L, 0);
  for (int t = 0; t < net.n_tensors; ++t) {
    std::vector<char> seen(L, 0);
    for (int l : net.labels[t]) {
      if (l < 0 || l >= L) fail(TNC_E_ARG, "tensor " + std::to_string(t) + ": label out of range");
      if (seen[l]) fail(TNC_E_ARG, "tensor " + std::to_string(t) + " repeats label " + std::to_string(l));
      seen[l] = 1;
      ++cnt[l];
    }
  }
  std::vector<char> is_open(L, 0);
  for (int l : net.open) {
    if (l < 0 || l >= L) fail(TNC_E_ARG, "open label out of range");
    if (is_open[l]) fail(TNC_E_ARG, "open list repeats label " + std::to_string(l));
    is_open[l] = 1;
  }
  net.kind.assign(L, LabelKind::Unused);
  net.user_batch.clear();
  for (int l = 0; l < L; ++l) {
    if (cnt[l] == 0) {
      if (is_open[l]) fail(TNC_E_ARG, "open label " + std::to_string(l) + " is on no tensor");
      continue;
    }
    if (is_open[l])
      net.kind[l] = cnt[l] == 1 ? LabelKind::Open : LabelKind::Batch;
    else if (cnt[l] == 2)
      net.kind[l] = LabelKind::Closed;
    else
      fail(TNC_E_ARG, "closed label " + std::to_string(l) + " is held by " + std::to_string(cnt[l]) +
                          " tensors (a closed label joins exactly two)");
  }
  for (int l : net.open)
    if (net.kind[l] == LabelKind::Batch) net.user_batch.push_back(l);
  net.numel.resize(net.n_tensors);
  net.stride.resize(net.n_tensors);
  for (int t = 0; t < net.n_tensors; ++t) {
    int64_t n = 1;
    std::vector<int64_t> ext;
    for (int l : net.labels[t]) {
      n = checked_mul(n, net.extents[l]);
      ext.push_back(net.extents[l]);
    }
    net.numel[t] = n;
    net.stride[t] = row_major(ext);
  }
}

void validate_path(const Net& net, const std::vector<std::array<int, 2>>& pairs) {
  const int n = net.n_tensors;
  if (n < 1) fail(TNC_E_ARG, "network has no tensors");
  if (static_cast<int>(pairs.size()) != n - 1)
    fail(TNC_E_PATH, "path has " + std::to_string(pairs.size()) + " steps; a tree over " + std::to_string(n) +
                         " leaves needs " + std::to_string(n - 1));
  std::vector<char> used(2 * n, 0);
  for (int s = 0; s < n - 1; ++s) {
    const int a = pairs[s][0], b = pairs[s][1];
    const int lim = n + s;
    if (a < 0 || b < 0 || a >= lim || b >= lim || a == b)
      fail(TNC_E_PATH, "step " + std::to_string(s) + ": operand id out of range");
    if (used[a] || used[b]) fail(TNC_E_PATH, "step " + std::to_string(s) + ": operand already consumed");
    used[a] = used[b] = 1;
  }
}

// ------------------------------------------------------------------ permutation tables
PermuteHost build_permute(const std::vector<int64_t>& ext0, const std::vector<int64_t>& st0) {
  PermuteHost P;
  // drop unit dims, fuse output-adjacent dims that are also input-adjacent
  std::vector<int64_t> ext, st;
  for (size_t j = 0; j < ext0.size(); ++j) {
    if (ext0[j] == 1) continue;
    if (!ext.empty() && st.back() == ext0[j] * st0[j]) {
      ext.back() *= ext0[j];
      st.back() = st0[j];
    } else {
      ext.push_back(ext0[j]);
      st.push_back(st0[j]);
    }
  }
  int64_t total = 1;
  for (int64_t e : ext) total *= e;
  if (static_cast<int>(ext.size()) > kMaxRank) fail(TNC_E_UNSUPPORTED, "permute rank above limit");
  GatherDesc& g = P.plain;
  std::memset(&g, 0, sizeof(g));
  g.total = total;
  g.rank = static_cast<int32_t>(ext.size());
  for (size_t j = 0; j < ext.size(); ++j) {
    g.ext[j] = ext[j];
    g.in_stride[j] = st[j];
  }
  auto plain_only = [&]() {
    PermuteHost Q;
    Q.plain = g;
    return Q;
  };
  if (total < 4096 || ext.size() <= 1) return P;

  // split a large dim at a divisor <= 64 so that tiles stay small
  auto split_dim = [&](size_t j) -> bool {
    int64_t e = ext[j];
    int64_t f = 0;
    for (int64_t c = 64; c >= 8; --c)
      if (e % c == 0) {
        f = c;
        break;
      }
    if (!f) return false;
    ext[j] = e / f;
    const int64_t s = st[j];
    st[j] = s * f;
    ext.insert(ext.begin() + j + 1, f);
    st.insert(st.begin() + j + 1, s);
    return true;
  };
  for (int guard = 0; guard < 16; ++guard) {
    const size_t r = ext.size();
    size_t fastest_in = 0;
    for (size_t j = 1; j < r; ++j)
      if (st[j] < st[fastest_in]) fastest_in = j;
    if (ext[fastest_in] > 64) {
      if (!split_dim(fastest_in)) return P;
      continue;
    }
    if (ext[r - 1] > 64) {
      if (!split_dim(r - 1)) return P;
      continue;
    }
    break;
  }
  const int r = static_cast<int>(ext.size());
  if (r > kMaxRank) return P;
  std::vector<int> by_stride(r);
  std::iota(by_stride.begin(), by_stride.end(), 0);
  std::sort(by_stride.begin(), by_stride.end(), [&](int a, int b) { return st[a] < st[b]; });
  // input-inner chain: the input's innermost modes, contiguous among themselves
  std::vector<char> inU(r, 0);
  std::vector<int> I;
  int64_t pI = 1;
  for (int idx = 0; idx < r && pI < 64; ++idx) {
    const int d = by_stride[idx];
    if (!I.empty()) {
      const int prev = I.back();
      if (st[d] != st[prev] * ext[prev]) break;
    }
    if (pI * ext[d] > 256) break;
    I.push_back(d);
    inU[d] = 1;
    pI *= ext[d];
  }
  int64_t T = pI, pO = 1;
  std::vector<int> O;
  for (int d = r - 1; d >= 0 && pO < 64; --d) {
    if (inU[d]) {
      O.push_back(d);
      pO *= ext[d];
      continue;
    }
    if (T * ext[d] > 4096) break;
    O.push_back(d);
    inU[d] = 1;
    pO *= ext[d];
    T *= ext[d];
  }
  if (T < 256 || pI < 8 || pO < 8) return P;  // no useful tile: plain gather
  // read order: I (fastest first), then U\I by output position (last fastest)
  std::vector<int> rfast;   // fastest first
  for (int d : I) rfast.push_back(d);
  for (int d = r - 1; d >= 0; --d)
    if (inU[d] && std::find(I.begin(), I.end(), d) == I.end()) rfast.push_back(d);
  // write order: O (output order, last fastest) then U\O by output position
  std::vector<int> wfast;
  for (int d : O) wfast.push_back(d);
  for (int d = r - 1; d >= 0; --d)
    if (inU[d] && std::find(O.begin(), O.end(), d) == O.end()) wfast.push_back(d);
  const std::vector<int64_t> ost = row_major(ext);
  std::vector<int64_t> rstride(r, 0);
  {
    int64_t s = 1;
    for (int d : rfast) {
      rstride[d] = s;
      s *= ext[d];
    }
  }
  auto pad = [](int64_t x) { return static_cast<int32_t>(x + (x >> 5)); };
  P.T = static_cast<int32_t>(T);
  P.slots = pad(T - 1) + 1;
  P.tile_in.resize(T);
  P.tile_slot_r.resize(T);
  P.tile_out.resize(T);
  P.tile_slot_w.resize(T);
  for (int64_t x = 0; x < T; ++x) {
    int64_t rest = x, in_off = 0;
    for (int d : rfast) {
      const int64_t dig = rest % ext[d];
      rest /= ext[d];
      in_off += dig * st[d];
    }
    if (in_off > INT32_MAX) return plain_only();
    P.tile_in[x] = static_cast<int32_t>(in_off);
    P.tile_slot_r[x] = pad(x);
    rest = x;
    int64_t out_off = 0, rpos = 0;
    for (int d : wfast) {
      const int64_t dig = rest % ext[d];
      rest /= ext[d];
      out_off += dig * ost[d];
      rpos += dig * rstride[d];
    }
    if (out_off > INT32_MAX) return plain_only();
    P.tile_out[x] = static_cast<int32_t>(out_off);
    P.tile_slot_w[x] = pad(rpos);
  }
  // outer dims (not in the tile), output order; split into lo (inner) and hi
  std::vector<int> outer;
  for (int d = 0; d < r; ++d)
    if (!inU[d]) outer.push_back(d);
  const int64_t n_tiles = total / T;
  int64_t L = 1;
  int split = static_cast<int>(outer.size());
  while (split > 0 && (L * ext[outer[split - 1]] <= 4096 || L * L < n_tiles)) {
    L *= ext[outer[split - 1]];
    --split;
  }
  auto make_tab = [&](int from, int to, std::vector<int64_t>& tab) {
    int64_t cnt = 1;
    for (int q = from; q < to; ++q) cnt *= ext[outer[q]];
    tab.assign(2 * cnt, 0);
    for (int64_t x = 0; x < cnt; ++x) {
      int64_t rest = x, io = 0, oo = 0;
      for (int q = to - 1; q >= from; --q) {
        const int d = outer[q];
        const int64_t dig = rest % ext[d];
        rest /= ext[d];
        io += dig * st[d];
        oo += dig * ost[d];
      }
      tab[2 * x] = io;
      tab[2 * x + 1] = oo;
    }
  };
  make_tab(split, static_cast<int>(outer.size()), P.lo_tab);
  make_tab(0, split, P.hi_tab);
  P.pairs = T % 2 == 0;
  for (int64_t x = 0; P.pairs && x < T; x += 2)
    P.pairs = P.tile_in[x] % 2 == 0 && P.tile_in[x + 1] == P.tile_in[x] + 1 && P.tile_out[x] % 2 == 0 &&
              P.tile_out[x + 1] == P.tile_out[x] + 1;
  for (size_t q = 0; P.pairs && q < P.lo_tab.size(); ++q) P.pairs = P.lo_tab[q] % 2 == 0;
  for (size_t q = 0; P.pairs && q < P.hi_tab.size(); ++q) P.pairs = P.hi_tab[q] % 2 == 0;
  P.L = static_cast<int32_t>(L);
  P.n_tiles = n_tiles;
  P.tiled = true;
  return P;
}

// ------------------------------------------------------------------ chunk plan
std::unique_ptr<ChunkPlan> build_chunk(const Plan& plan, int j) {
  const Net& net = *plan.net;
  auto cp = std::make_unique<ChunkPlan>();
  cp->j = j;
  cp->hs = plan.suffix_prod[j];
  const int L = static_cast<int>(net.extents.size());
  const int n = net.n_tensors;
  const int ns = static_cast<int>(plan.pairs.size());
  const int n_ids = n + ns;
  const int nS = static_cast<int>(plan.sliced.size());
  std::vector<char> removed(L, 0), is_batch(L, 0), is_open(L, 0);
  for (int i = 0; i < nS - j; ++i) removed[plan.sliced[i]] = 1;
  for (int i = nS - j; i < nS; ++i) cp->batch.push_back(plan.sliced[i]);
  for (int l : net.user_batch) cp->batch.push_back(l);
  for (int l : cp->batch) is_batch[l] = 1;
  for (int l : net.open) is_open[l] = 1;

  // forward: label sets of every id, labels summed at each step
  std::vector<std::vector<int>> sets(n_ids);
  std::vector<int> live(L, 0);
  for (int t = 0; t < n; ++t)
    for (int l : net.labels[t])
      if (!removed[l]) {
        sets[t].push_back(l);
        ++live[l];
      }
  std::vector<std::vector<int>> summed(ns);
  std::vector<int> consumer(n_ids, ns);
  std::vector<int> mark(L, -1);
  for (int s = 0; s < ns; ++s) {
    const int a = plan.pairs[s][0], b = plan.pairs[s][1];
    consumer[a] = consumer[b] = s;
    for (int l : sets[a]) mark[l] = s;
    std::vector<int> out;
    for (int l : sets[a]) out.push_back(l);
    for (int l : sets[b]) {
      if (mark[l] == s) {  // shared
        const bool keep = is_batch[l] || is_open[l] || live[l] > 2;
        if (keep) {
          live[l] -= 1;
        } else {
          live[l] -= 2;
          summed[s].push_back(l);
        }
      } else {
        out.push_back(l);
      }
    }
    std::sort(summed[s].begin(), summed[s].end());
    for (int l : summed[s]) mark[l] = -2;  // drop from out
    std::vector<int> out2;
    for (int l : out)
      if (!(mark[l] == -2)) out2.push_back(l);
    for (int l : summed[s]) mark[l] = -1;
    for (int l : sets[a]) mark[l] = -1;
    sets[n + s] = std::move(out2);
  }
  const int root = ns > 0 ? n + ns - 1 : 0;
  cp->root_id = root;

  // backward pass (Sec. IV-A): output order known, operands get
  // [kept labels in output order || labels summed here (ascending)]
  cp->order.assign(n_ids, {});
  {
    std::vector<char> in_root(L, 0);
    for (int l : sets[root]) in_root[l] = 1;
    for (int l : cp->batch)
      if (in_root[l]) cp->order[root].push_back(l);
    for (int l : net.open)
      if (in_root[l] && !is_batch[l]) cp->order[root].push_back(l);
    if (cp->order[root].size() != sets[root].size()) fail(TNC_E_ARG, "root labels differ from the open labels");
  }
  cp->steps.resize(ns);
  std::vector<int> owner(L, -1);
  for (int s = ns - 1; s >= 0; --s) {
    const int c = n + s;
    int a = plan.pairs[s][0], b = plan.pairs[s][1];
    const std::vector<int>& tc = cp->order[c];
    for (int l : sets[a]) owner[l] = a;
    for (int l : sets[b])
      if (owner[l] != a) owner[l] = b;
    // orientation: the output's innermost non-batch label goes to the N side
    for (int q = static_cast<int>(tc.size()) - 1; q >= 0; --q) {
      if (is_batch[tc[q]]) continue;
      if (owner[tc[q]] == a) std::swap(a, b);
      break;
    }
    StepPlan& sp = cp->steps[s];
    sp.A = a;
    sp.B = b;
    sp.C = c;
    std::vector<char> inA(L, 0), inB(L, 0);
    for (int l : sets[a]) inA[l] = 1;
    for (int l : sets[b]) inB[l] = 1;
    for (int l : tc) {
      if (is_batch[l])
        sp.H.push_back(l);
      else if (inA[l])
        sp.M.push_back(l);
      else
        sp.N.push_back(l);
    }
    sp.K = summed[s];
    for (int x : {a, b}) {
      std::vector<int>& o = cp->order[x];
      o.clear();
      const std::vector<char>& in = x == a ? inA : inB;
      for (int l : tc)
        if (in[l]) o.push_back(l);
      for (int l : sp.K) o.push_back(l);
    }
    std::vector<int> nat = sp.H;
    nat.insert(nat.end(), sp.M.begin(), sp.M.end());
    nat.insert(nat.end(), sp.N.begin(), sp.N.end());
    sp.natural = nat == tc;
    for (int l : sets[a]) owner[l] = -1;
    for (int l : sets[b]) owner[l] = -1;
  }
  // sizes
  cp->numel.assign(n_ids, 1);
  for (int id = 0; id < n_ids; ++id)
    for (int l : cp->order[id]) cp->numel[id] = checked_mul(cp->numel[id], net.extents[l]);
  for (int id = 0; id < n_ids; ++id) cp->max_tensor = std::max(cp->max_tensor, cp->numel[id]);

  // leaves: direct use or a gather-permute into the arena
  cp->leaf.resize(n);
  cp->tensor_buf.assign(n_ids, -1);
  int n_slots = 0;
  for (int t = 0; t < n; ++t) {
    LeafPrep& lp = cp->leaf[t];
    lp.leaf = t;
    lp.step = consumer[t] < ns ? consumer[t] : 0;
    const std::vector<int>& stored = net.labels[t];
    std::vector<int> kept;
    for (size_t q = 0; q < stored.size(); ++q) {
      if (removed[stored[q]])
        lp.fixed.emplace_back(stored[q], net.stride[t][q]);
      else
        kept.push_back(stored[q]);
    }
    lp.direct = lp.fixed.empty() && kept == cp->order[t];
    if (lp.direct) continue;
    std::unordered_map<int, int64_t> sof;
    for (size_t q = 0; q < stored.size(); ++q) sof[stored[q]] = net.stride[t][q];
    std::vector<int64_t> ext, ist;
    for (int l : cp->order[t]) {
      ext.push_back(net.extents[l]);
      ist.push_back(sof[l]);
    }
    lp.perm = build_permute(ext, ist);
    if (!lp.fixed.empty()) lp.base_slot = n_slots++;
    cp->n_permutes++;
    cp->transpose_bytes += 16.0 * static_cast<double>(cp->numel[t]);
  }
  cp->n_base_slots = n_slots;
  // leaves without a per-chunk base offset are the same in every run: up to
  // 2^22 elements each they are permuted once into the leaf cache (not the
  // leaves a batcher rewrites before every run)
  constexpr int64_t kCacheLeafElems = int64_t{1} << 22;
  for (int t = 0; t < n && ns > 0; ++t) {
    LeafPrep& lp = cp->leaf[t];
    if (lp.direct || lp.base_slot >= 0 || cp->numel[t] > kCacheLeafElems) continue;
    if (!plan.volatile_leaf.empty() && plan.volatile_leaf[t]) continue;
    lp.cached = true;
    lp.cache_off = cp->cache_bytes;
    cp->cache_bytes += align_up(cp->numel[t] * 8);
    cp->n_cached++;
  }
  for (int t = 0; t < n; ++t)
    if (!cp->leaf[t].direct && !cp->leaf[t].cached && ns > 0) cp->steps[cp->leaf[t].step].preps.push_back(t);

  // steps: sizes, batch strides, kernel, output offsets
  for (int s = 0; s < ns; ++s) {
    StepPlan& sp = cp->steps[s];
    auto prod = [&](const std::vector<int>& ls) {
      int64_t p = 1;
      for (int l : ls) p *= net.extents[l];
      return p;
    };
    sp.h = prod(sp.H);
    sp.m = prod(sp.M);
    sp.n = prod(sp.N);
    sp.k = prod(sp.K);
    // A leaf whose sliced labels are fixed per chunk would be gathered into
    // the arena before every batch; when this step runs one thread per
    // output (no transposed launch), it is read in place instead: its own
    // strides, row and K offset tables, and the chunk's base offset.
    const bool small_step = choose_gemm_kernel(sp.h, sp.m, sp.n, sp.k) == GemmKernel::SMALL &&
                            choose_gemm_kernel(sp.h, sp.n, sp.m, sp.k) != GemmKernel::MFMA;
    for (int x : {sp.A, sp.B})
      if (x < n && small_step && cp->leaf[x].base_slot >= 0 && !cp->leaf[x].inplace) {
        cp->leaf[x].inplace = true;
        cp->n_permutes--;
        cp->transpose_bytes -= 16.0 * static_cast<double>(cp->numel[x]);
        auto& pr = sp.preps;
        pr.erase(std::remove(pr.begin(), pr.end(), x), pr.end());
      }
    auto strides_of = [&](int id) {
      std::unordered_map<int, int64_t> m;
      if (id < n && cp->leaf[id].inplace) {  // the leaf's own strides (fixed labels dropped)
        const std::vector<int>& stored = net.labels[id];
        for (size_t q = 0; q < stored.size(); ++q)
          if (!removed[stored[q]]) m[stored[q]] = net.stride[id][q];
        return m;
      }
      const std::vector<int>& o = cp->order[id];
      int64_t s2 = 1;
      for (int q = static_cast<int>(o.size()) - 1; q >= 0; --q) {
        m[o[q]] = s2;
        s2 *= net.extents[o[q]];
      }
      return m;
    };
    const auto sa = strides_of(sp.A), sb = strides_of(sp.B), sc = strides_of(sp.C);
    sp.hA = 1;
    sp.hB = 1;
    std::vector<int64_t> bext, bsa, bsb;
    for (int l : sp.H) {
      const auto ia = sa.find(l), ib = sb.find(l);
      if (ia != sa.end()) sp.hA *= net.extents[l];
      if (ib != sb.end()) sp.hB *= net.extents[l];
      bext.push_back(net.extents[l]);
      bsa.push_back(ia != sa.end() ? ia->second : 0);
      bsb.push_back(ib != sb.end() ? ib->second : 0);
    }
    // merge batch dims that are contiguous in both operands
    std::vector<int64_t> me, ma, mb;
    for (size_t q = 0; q < bext.size(); ++q) {
      if (bext[q] == 1) continue;
      if (!me.empty() && ma.back() == bext[q] * bsa[q] && mb.back() == bext[q] * bsb[q]) {
        me.back() *= bext[q];
        ma.back() = bsa[q];
        mb.back() = bsb[q];
      } else {
        me.push_back(bext[q]);
        ma.push_back(bsa[q]);
        mb.push_back(bsb[q]);
      }
    }
    if (static_cast<int>(me.size()) > kMaxBatchDims) fail(TNC_E_UNSUPPORTED, "too many batch dims");
    // launch orientation: transposed (B as the row operand) when only that
    // orientation reaches MFMA, or when it pads the 64 x 32 wave tiles less
    auto waste = [](int64_t r, int64_t c) {
      return static_cast<double>((r + 63) / 64 * 64) / r * static_cast<double>((c + 31) / 32 * 32) / c;
    };
    const GemmKernel k0 = choose_gemm_kernel(sp.h, sp.m, sp.n, sp.k);
    const GemmKernel k1 = choose_gemm_kernel(sp.h, sp.n, sp.m, sp.k);
    sp.swap = k1 == GemmKernel::MFMA && (k0 != GemmKernel::MFMA || waste(sp.n, sp.m) < waste(sp.m, sp.n));
    sp.kind = sp.swap ? k1 : k0;
    sp.la = sp.swap ? sp.B : sp.A;
    sp.lb = sp.swap ? sp.A : sp.B;
    sp.lm = sp.swap ? sp.n : sp.m;
    sp.ln = sp.swap ? sp.m : sp.n;
    if (sp.swap) std::swap(ma, mb);
    GemmDesc& d = sp.desc;
    std::memset(&d, 0, sizeof(d));
    d.m = sp.lm;
    d.n = sp.ln;
    d.k = sp.k;
    d.h = sp.h;
    d.nbd = static_cast<int32_t>(me.size());
    d.pow2 = 1;
    for (size_t q = 0; q < me.size(); ++q) {
      if (me[q] > INT32_MAX) fail(TNC_E_UNSUPPORTED, "batch extent too large");
      d.bext[q] = static_cast<int32_t>(me[q]);
      d.bsA[q] = ma[q];
      d.bsB[q] = mb[q];
      int sh = 0;
      while ((int64_t{1} << sh) < me[q]) ++sh;
      d.bshift[q] = sh;
      if ((int64_t{1} << sh) != me[q]) d.pow2 = 0;
    }
    // operand tables of in-place leaves: row i (digits over the operand's
    // kept labels in the output's order) and K index l (digits over K)
    auto table = [&](const std::vector<int>& ls, const std::unordered_map<int, int64_t>& st) {
      int64_t cnt = 1;
      for (int l : ls) cnt *= net.extents[l];
      std::vector<int64_t> off(cnt);
      for (int64_t i = 0; i < cnt; ++i) {
        int64_t rest = i, o = 0;
        for (int q = static_cast<int>(ls.size()) - 1; q >= 0; --q) {
          const int64_t e = net.extents[ls[q]];
          o += (rest % e) * st.at(ls[q]);
          rest /= e;
        }
        off[i] = o;
      }
      return off;
    };
    if (sp.la < n && cp->leaf[sp.la].inplace) {
      sp.tab[0] = table(sp.swap ? sp.N : sp.M, sp.swap ? sb : sa);
      sp.tab[1] = table(sp.K, sp.swap ? sb : sa);
    }
    if (sp.lb < n && cp->leaf[sp.lb].inplace) {
      sp.tab[2] = table(sp.swap ? sp.M : sp.N, sp.swap ? sa : sb);
      sp.tab[3] = table(sp.K, sp.swap ? sa : sb);
    }
    // store tables (launch orientation) for permuted or transposed stores
    if (!sp.natural || sp.swap) {
      std::vector<int64_t> tm(sp.m), tn(sp.n);
      auto fill = [&](const std::vector<int>& ls, std::vector<int64_t>& off) {
        for (int64_t i = 0; i < static_cast<int64_t>(off.size()); ++i) {
          int64_t rest = i, o = 0;
          for (int q = static_cast<int>(ls.size()) - 1; q >= 0; --q) {
            const int64_t e = net.extents[ls[q]];
            o += (rest % e) * sc.at(ls[q]);
            rest /= e;
          }
          off[i] = o;
        }
      };
      fill(sp.M, tm);
      fill(sp.N, tn);
      sp.offM = sp.swap ? std::move(tn) : std::move(tm);
      sp.offN = sp.swap ? std::move(tm) : std::move(tn);
    }
    if (!sp.natural) cp->n_perm_stores++;
    // split K when the output alone cannot fill the chip: the K range is cut
    // into S equal parts (one more batch dim), partial products go to an
    // arena scratch buffer and the split-K epilogue sums them in order
    int64_t S = 1;
    if (sp.kind == GemmKernel::MFMA) {
      const int64_t t0 = sp.h * ((sp.lm + 127) / 128) * ((sp.ln + 63) / 64);
      // parts of at least 8 K stages (128 complex); a long K on few tiles is
      // a long serial loop on few CUs, whatever the step's size
      if (t0 < 512 && sp.k >= 256)
        while (t0 * S * 2 <= 2048 && sp.k / (S * 2) >= 128 && sp.k % (16 * S * 2) == 0) S *= 2;
    } else if (sp.kind == GemmKernel::DOT) {
      const int64_t outs = sp.h * sp.lm * sp.ln;
      if (outs < 4096 && sp.k >= 8192)
        while (outs * S * 2 <= 16384 && sp.k / (S * 2) >= 1024 && sp.k % (S * 2) == 0) S *= 2;
    }
    if (S > 1 && d.nbd < kMaxBatchDims) {
      const int q = d.nbd++;
      d.bext[q] = static_cast<int32_t>(S);
      d.bsA[q] = sp.k / S;
      d.bsB[q] = sp.k / S;
      int sh = 0;
      while ((int64_t{1} << sh) < S) ++sh;
      d.bshift[q] = sh;
      d.h = sp.h * S;
      d.k = sp.k / S;
      d.ldk = sp.k;
      sp.split = static_cast<int>(S);
    }
    // the fallback the permuted-store epilogue replaces: store in the launch
    // order and transpose into the consumer's order with a separate
    // permutation (split-K steps keep their epilogue, itself a separate pass)
    if (plan.store_order == 1 && !sp.natural && sp.split == 1) {
      sp.trans = true;
      sp.offM.clear();
      sp.offN.clear();
      const std::vector<int>& rows = sp.swap ? sp.N : sp.M;
      const std::vector<int>& cols = sp.swap ? sp.M : sp.N;
      std::unordered_map<int, int64_t> ts;   // stride of each label in [H | rows | cols]
      int64_t st = 1;
      for (int q = static_cast<int>(cols.size()) - 1; q >= 0; --q) {
        ts[cols[q]] = st;
        st *= net.extents[cols[q]];
      }
      for (int q = static_cast<int>(rows.size()) - 1; q >= 0; --q) {
        ts[rows[q]] = st;
        st *= net.extents[rows[q]];
      }
      for (int q = static_cast<int>(sp.H.size()) - 1; q >= 0; --q) {
        ts[sp.H[q]] = st;
        st *= net.extents[sp.H[q]];
      }
      std::vector<int64_t> ext, ist;
      for (int l : cp->order[sp.C]) {
        ext.push_back(net.extents[l]);
        ist.push_back(ts.at(l));
      }
      sp.tperm = build_permute(ext, ist);
    }
    // split precision on large single GEMMs: split each operand once into
    // bf16 planes (4M form: 8 + 8 bytes per element of A, 8 + 16 of B moved,
    // about 1 % of the GEMM's time from 4096 x 4096 up; 3M form: 8 + 12 per
    // element of each operand, plus its three float32 products' 12 + 12 + 8
    // per output element) rather than in the staging of every workgroup
    // that reads it
    sp.presplit = plan.prec == TNC_PREC_BF16X3 && sp.kind == GemmKernel::MFMA && sp.split == 1 && !sp.trans &&
                  d.h == 1 && sp.lm >= 4096 && sp.ln >= 4096;
    // an operand leaf that is permuted anyway writes the planes itself (the
    // permute and the split in one pass) when rows are whole blocks: 16 k
    // in the 4M form, 32 real k (2 x 16 pairs) in the 3M form
    if (sp.presplit && sp.k % (plan.form == TNC_GEMM_3M ? 32 : 16) == 0 && row_stride(d) == sp.k)
      for (int side = 1; side <= 2; ++side) {
        const int id = side == 1 ? sp.la : sp.lb;
        if (id >= n) continue;
        LeafPrep& lp = cp->leaf[id];
        if (!lp.direct && !lp.cached && !lp.inplace && lp.perm.tiled) lp.planes_side = side;
      }
    cp->flops += 8.0 * static_cast<double>(sp.h) * sp.m * sp.n * sp.k;
    cp->bytes += 8.0 * (static_cast<double>(sp.hA) * sp.m * sp.k + static_cast<double>(sp.hB) * sp.n * sp.k +
                        static_cast<double>(sp.h) * sp.m * sp.n);
  }

  // execution order: step by step, or level by level of the tree (a step's
  // level is one more than its operands'; all steps of a level are
  // independent and run together)
  std::vector<int> lvl(n_ids, 0);
  for (int s = 0; s < ns; ++s) lvl[n + s] = 1 + std::max(lvl[plan.pairs[s][0]], lvl[plan.pairs[s][1]]);
  cp->grouped = plan.grouping != 0 && ns > 0;
  auto when = [&](int s) { return cp->grouped ? lvl[n + s] : s; };
  const int t_end = ns == 0 ? 0 : (cp->grouped ? lvl[root] + 1 : ns);
  if (cp->grouped) {
    cp->levels.assign(lvl[root] + 1, LevelPlan{});
    for (int s = 0; s < ns; ++s) {
      LevelPlan& level = cp->levels[lvl[n + s]];
      const StepPlan& sp = cp->steps[s];
      if (sp.kind == GemmKernel::SMALL && n + s != root && !sp.trans)
        level.group_steps.push_back(s);
      else
        level.single_steps.push_back(s);
      for (int t : sp.preps) {
        const LeafPrep& lp = cp->leaf[t];
        if (!lp.perm.tiled && lp.perm.plain.rank <= kGroupRank)
          level.group_leaves.push_back(t);
        else
          level.single_leaves.push_back(t);
      }
    }
  }

  // arena buffers: live ranges in execution time, first fit by decreasing size
  struct Iv {
    int64_t bytes;
    int t0, t1;
    int id;
  };
  std::vector<Iv> ivs;
  for (int t = 0; t < n; ++t) {
    if (cp->leaf[t].direct || cp->leaf[t].cached || cp->leaf[t].inplace) continue;
    const int tt = ns > 0 ? when(cp->leaf[t].step) : 0;
    ivs.push_back({align_up(cp->numel[t] * 8), tt, t == root ? t_end : tt, t});
  }
  for (int s = 0; s < ns; ++s) {
    const int c = n + s;
    ivs.push_back({align_up(cp->numel[c] * 8), when(s), consumer[c] < ns ? when(consumer[c]) : t_end, c});
    const StepPlan& sp = cp->steps[s];
    if (sp.split > 1 || sp.trans)  // split-K partials or the untransposed output, live during the step only
      ivs.push_back({align_up(sp.h * sp.split * sp.lm * sp.ln * 8), when(s), when(s), -1 - s});
    if (sp.presplit)  // the operands' bf16 planes (and the 3M products), live during the step only
      ivs.push_back({align_up(plan.form == TNC_GEMM_3M ? presplit_3m_layout(sp.lm, sp.ln, sp.k).bytes
                                                       : static_cast<int64_t>(presplit_plane_bytes(sp.lm, sp.ln, sp.k))),
                     when(s), when(s), -1 - ns - s});
  }
  std::vector<int> idx(ivs.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) {
    if (ivs[x].bytes != ivs[y].bytes) return ivs[x].bytes > ivs[y].bytes;
    return ivs[x].t0 < ivs[y].t0;
  });
  cp->buf_bytes.resize(ivs.size());
  cp->buf_off.assign(ivs.size(), 0);
  std::vector<int> placed;
  int64_t peak = 0;
  for (int x : idx) {
    std::vector<std::pair<int64_t, int64_t>> busy;
    for (int y : placed)
      if (!(ivs[y].t1 < ivs[x].t0 || ivs[x].t1 < ivs[y].t0)) busy.emplace_back(cp->buf_off[y], cp->buf_off[y] + ivs[y].bytes);
    std::sort(busy.begin(), busy.end());
    int64_t off = 0;
    for (auto& b : busy) {
      if (off + ivs[x].bytes <= b.first) break;
      off = std::max(off, b.second);
    }
    cp->buf_off[x] = off;
    cp->buf_bytes[x] = ivs[x].bytes;
    peak = std::max(peak, off + ivs[x].bytes);
    placed.push_back(x);
  }
  for (size_t q = 0; q < ivs.size(); ++q) {
    const int id = ivs[q].id;
    if (id < 0) {
      const int s = -1 - id;
      if (s < ns)
        cp->steps[s].scratch_buf = static_cast<int>(q);
      else
        cp->steps[s - ns].presplit_buf = static_cast<int>(q);
      continue;
    }
    cp->tensor_buf[id] = static_cast<int>(q);
    if (id < n) cp->leaf[id].buf = static_cast<int>(q);
  }
  cp->peak = peak;

  // result: root minus the slice batch labels; map to the user's open order
  cp->R = cp->numel[root] / cp->hs;
  std::vector<int> reduced(cp->order[root].begin() + j, cp->order[root].end());
  if (reduced != net.open) {
    std::vector<int64_t> ext;
    for (int l : reduced) ext.push_back(net.extents[l]);
    const auto rst = row_major(ext);
    std::unordered_map<int, int64_t> pos;
    for (size_t q = 0; q < reduced.size(); ++q) pos[reduced[q]] = rst[q];
    cp->result_perm.resize(cp->R);
    for (int64_t u = 0; u < cp->R; ++u) {
      int64_t rest = u, o = 0;
      for (int q = static_cast<int>(net.open.size()) - 1; q >= 0; --q) {
        const int l = net.open[q];
        o += (rest % net.extents[l]) * pos[l];
        rest /= net.extents[l];
      }
      cp->result_perm[u] = o;
    }
  }
  assign_variants(plan, *cp, false);
  return cp;
}

// extra run workspace after the intermediates: per-chunk base offsets
size_t run_extra_bytes(const ChunkPlan& cp, int64_t n_chunks) {
  return static_cast<size_t>(align_up(std::max<int64_t>(1, n_chunks) * std::max(1, cp.n_base_slots) * 8));
}

void choose_chunking(Plan& plan, size_t budget) {
  const int nS = static_cast<int>(plan.sliced.size());
  plan.chunks.clear();
  plan.chunks.resize(nS + 1);
  plan.chunks[0] = build_chunk(plan, 0);
  int best = 0;
  for (int j = 1; j <= nS; ++j) {
    if (plan.max_chunk_user > 0 && plan.suffix_prod[j] > plan.max_chunk_user) break;
    auto cp = build_chunk(plan, j);
    const size_t need = static_cast<size_t>(cp->peak) + run_extra_bytes(*cp, 1);
    if (budget && need > budget) break;
    plan.chunks[j] = std::move(cp);
    best = j;
  }
  plan.j_max = best;
}

ChunkPlan& Plan::chunk(int j) {
  std::lock_guard<std::mutex> g(mu);
  if (!chunks[j]) chunks[j] = build_chunk(*this, j);
  return *chunks[j];
}

}  // namespace tnc
