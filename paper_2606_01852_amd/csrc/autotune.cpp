// Autotuner for the MFMA tile variant of each GEMM step (an extension; the
// paper leaves each step's kernel to its library).
//
// For every distinct step shape (precision, form, output store, h, m, n, k)
// the candidate workgroup shapes are timed with HIP events on a stand-in
// problem of the same structure, filled with hashed uniform values (m, then
// K down to 8192, then the batch cut so that a trial stays near 2e13 FLOP
// while keeping enough tiles to show the step's wave quantization), and the
// fastest is kept.  Choices live in a per-context cache, optionally backed
// by a text file (TNC_AUTOTUNE_CACHE) so later processes skip the timing.
// Without tuning a shape-based default is used.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "core.hpp"

namespace tnc {

namespace {

int64_t tiles_for(int variant, int64_t h, int64_t m, int64_t n) {
  int bm = 0, bnc = 0;
  gemm_variant_tile(variant, &bm, &bnc);
  return h * ((m + bm - 1) / bm) * ((n + bnc - 1) / bnc);
}

double padding_waste(int variant, int64_t m, int64_t n) {
  int bm = 0, bnc = 0;
  gemm_variant_tile(variant, &bm, &bnc);
  const double pm = static_cast<double>((m + bm - 1) / bm * bm);
  const double pn = static_cast<double>((n + bnc - 1) / bnc * bnc);
  return 1.0 - static_cast<double>(m) * n / (pm * pn);
}

// Ranking of the variants by measured per-tile throughput on large shapes.
const std::vector<int>& ranking(tnc_prec prec, tnc_cgemm form) {
  static const std::vector<int> r4m = {3, 2, 0, 1, 4, 5, 6};
  static const std::vector<int> r3m = {0, 2, 4, 1, 5, 6};  // 0: three (2,2) workgroups per CU
  static const std::vector<int> rbf = {3, 0, 2, 1, 4, 5, 6};  // 3: the wide-wave 256 x 128 tile
  if (form == TNC_GEMM_3M) return r3m;  // complex64 and split precision alike
  return prec == TNC_PREC_BF16X3 ? rbf : r4m;
}

std::vector<int> candidates(tnc_prec prec, tnc_cgemm form, int64_t h, int64_t m, int64_t n) {
  std::vector<int> out;
  for (int v : ranking(prec, form))
    if (tiles_for(v, h, m, n) * 64 < (int64_t{1} << 32) && padding_waste(v, m, n) < 0.5) out.push_back(v);
  if (out.empty()) out.push_back(0);
  return out;
}

}  // namespace

int default_variant(tnc_prec prec, tnc_cgemm form, int64_t h, int64_t m, int64_t n) {
  // the best-ranked shape that still gives every CU a few tiles and wastes
  // little on padding; small problems fall through to the small shapes
  for (int v : ranking(prec, form))
    if (tiles_for(v, h, m, n) >= 4 * 256 && padding_waste(v, m, n) <= 0.125) return v;
  return 4;
}

std::string TuneKey::str() const {
  std::ostringstream o;
  o << prec << ' ' << form << ' ' << perm << ' ' << h << ' ' << m << ' ' << n << ' ' << k;
  return o.str();
}

void load_tune_cache(Ctx& c) {
  const char* path = std::getenv("TNC_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  TuneKey key;
  int v = 0;
  while (f >> key.prec >> key.form >> key.perm >> key.h >> key.m >> key.n >> key.k >> v)
    if (v >= 0 && v < kGemmVariants) c.tune_cache[key] = v;
}

static void save_tune_entry(const TuneKey& key, int v) {
  const char* path = std::getenv("TNC_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key.str() << ' ' << v << '\n';
}

int tune_shape(Ctx& c, const TuneKey& key, int64_t k, bool perm_store) {
  {
    std::lock_guard<std::mutex> g(c.tune_mu);
    auto it = c.tune_cache.find(key);
    if (it != c.tune_cache.end()) return it->second;
  }
  const tnc_prec prec = static_cast<tnc_prec>(key.prec);
  const tnc_cgemm form = static_cast<tnc_cgemm>(key.form);
  const std::vector<int> cand = candidates(prec, form, key.h, key.m, key.n);
  int best = cand.front();
  if (cand.size() > 1) {
    // stand-in problem near 2e13 FLOP (about 0.15 s).  m is cut first while
    // the grid keeps 8 or more rounds of the largest workgroup (256 x 128)
    // over the 256 CUs, so wave quantization -- which separates the shapes on
    // few-tile steps -- stays that of the step; K stays whole there, since
    // whether a K panel fits an XCD's 4 MiB L2 also ranks the shapes (3M
    // (2,2) leads (2,4) at k = 2048 and trails it by 5 % at k = 16384).
    // Then K (down to 8192), the batch, and m below that bound.
    int64_t h = key.h, m = key.m;
    const double target = 2e13;
    auto flop = [&] { return 8.0 * h * m * key.n * k; };
    auto half_m = [](int64_t x) { return (x / 2 + 255) / 256 * 256; };
    while (m > 8192 && flop() > target && h * ((half_m(m) + 255) / 256) * ((key.n + 127) / 128) >= 2048)
      m = half_m(m);
    while (k > 8192 && k % 32 == 0 && flop() > target) k /= 2;
    while (h > 1 && flop() > target) h = (h + 1) / 2;
    while (m > 4096 && flop() > target) m = half_m(m);
    // and its operands stay within 8 GiB beside the caller's arena (the
    // batch shrinks; 2048 or more tiles remain for batches of this size)
    auto bytes = [&] { return 8.0 * h * (m * k + key.n * k + m * key.n); };
    while (h > 1 && bytes() > 8.0 * (int64_t{1} << 30)) h = (h + 1) / 2;
    DeviceBuf a, b, cc, offm, offn;
    a.alloc(static_cast<size_t>(h * m * k) * 8);
    b.alloc(static_cast<size_t>(h * key.n * k) * 8);
    cc.alloc(static_cast<size_t>(h * m * key.n) * 8);
    check_hip(launch_fill_hash(static_cast<float*>(a.ptr), h * m * k * 2, 0x5eed0001u, c.stream), "tune fill");
    check_hip(launch_fill_hash(static_cast<float*>(b.ptr), h * key.n * k * 2, 0x5eed0002u, c.stream), "tune fill");
    GemmDesc d;
    std::memset(&d, 0, sizeof(d));
    d.A = static_cast<const float2*>(a.ptr);
    d.B = static_cast<const float2*>(b.ptr);
    d.C = static_cast<float2*>(cc.ptr);
    d.m = m;
    d.n = key.n;
    d.k = k;
    d.h = h;
    if (h > 1) {
      d.nbd = 1;
      d.bext[0] = static_cast<int32_t>(h);
      d.bsA[0] = m * k;
      d.bsB[0] = key.n * k;
      d.pow2 = 0;
    }
    if (perm_store) {  // a permuted store with the natural offsets: same access count
      std::vector<int64_t> om(m), on(key.n);
      for (int64_t i = 0; i < m; ++i) om[i] = i * key.n;
      for (int64_t j = 0; j < key.n; ++j) on[j] = j;
      offm.alloc(om.size() * 8);
      offn.alloc(on.size() * 8);
      check_hip(hipMemcpy(offm.ptr, om.data(), om.size() * 8, hipMemcpyHostToDevice), "tune tables");
      check_hip(hipMemcpy(offn.ptr, on.data(), on.size() * 8, hipMemcpyHostToDevice), "tune tables");
      d.offM = static_cast<const int64_t*>(offm.ptr);
      d.offN = static_cast<const int64_t*>(offn.ptr);
    }
    const Form f = form == TNC_GEMM_3M ? Form::M3 : Form::M4;
    const Prec p = prec == TNC_PREC_BF16X3 ? Prec::BF16X3 : Prec::C64;
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "event");
    check_hip(hipEventCreate(&e1), "event");
    float best_ms = 1e30f;
    for (int v : cand) {
      check_hip(launch_gemm(d, GemmKernel::MFMA, v, f, p, c.stream), "tune launch");  // warm-up
      check_hip(hipEventRecord(e0, c.stream), "event");
      for (int r = 0; r < 2; ++r) check_hip(launch_gemm(d, GemmKernel::MFMA, v, f, p, c.stream), "tune launch");
      check_hip(hipEventRecord(e1, c.stream), "event");
      check_hip(hipEventSynchronize(e1), "event");
      float ms = 0;
      check_hip(hipEventElapsedTime(&ms, e0, e1), "event");
      // candidates come in ranking order (full-size sweeps); a later one
      // must win by more than 1 %, the spread of repeated trials
      if (ms < 0.99f * best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  {
    std::lock_guard<std::mutex> g(c.tune_mu);
    c.tune_cache[key] = best;
  }
  save_tune_entry(key, best);
  return best;
}

void assign_variants(const Plan& plan, ChunkPlan& cp, bool tune) {
  Ctx& c = *plan.net->ctx;
  for (StepPlan& sp : cp.steps) {
    if (sp.kind != GemmKernel::MFMA) continue;
    const GemmDesc& d = sp.desc;
    const bool perm = !sp.offM.empty() && sp.split == 1;
    const TuneKey key{static_cast<int>(plan.prec), static_cast<int>(plan.form), perm ? 1 : 0, d.h, d.m, d.n, d.k};
    bool cached = false;
    {
      std::lock_guard<std::mutex> g(c.tune_mu);
      auto it = c.tune_cache.find(key);
      if (it != c.tune_cache.end()) {
        sp.variant = it->second;
        cached = true;
      }
    }
    if (cached) continue;
    if (tune && !c.host_only)
      sp.variant = tune_shape(c, key, d.k, perm);
    else
      sp.variant = default_variant(plan.prec, plan.form, d.h, d.m, d.n);
  }
}

}  // namespace tnc
