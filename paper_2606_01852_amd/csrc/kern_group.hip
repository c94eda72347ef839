// Grouped launches: every small step (or leaf gather) of one level of the
// contraction tree (the SSA path of Sec. II-B) in a single kernel.
//
// Steps of one level depend only on lower levels, so they can run together.
// Circuit and grid networks have hundreds of tiny steps but trees only
// 10-20 levels deep; one launch per level instead of per step removes most
// of the launch chain that otherwise bounds their latency.  Each thread
// finds its step by binary search over the level's prefix sums of work items
// and then does exactly what the one-step kernel does for that element, so
// results are bitwise those of the per-step launches.  The "runs" forms do
// the same over the levels of several runs of one structure (a fused
// serving job): a thread first finds its run, then its step in that run's
// own table.
#include "gemm_common.hpp"

namespace tnc {

namespace {

__device__ __forceinline__ int find_item(const int64_t* prefix, int n, int64_t gt) {
  int lo = 0, hi = n - 1;  // largest i with prefix[i] <= gt
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= gt)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ T* reloc(const void* p, int flag, char* arena) {
  return flag ? reinterpret_cast<T*>(arena + reinterpret_cast<intptr_t>(p)) : (T*)p;
}

// Work item gt of a level's grouped small GEMMs: one output element.
template <bool SPLIT>
__device__ __forceinline__ void small_gemm_item(const GroupGemm* __restrict__ g, const int64_t* __restrict__ prefix,
                                                int n, int64_t gt, char* arena, const int64_t* bases) {
  const int s = find_item(prefix, n, gt);
  const GroupGemm& e = g[s];
  const GemmDesc& d = e.d;
  const int64_t idx = gt - prefix[s];
  const int64_t mn = d.m * d.n;
  const int64_t b = idx / mn;
  const int64_t r = idx - b * mn;
  const int64_t i = r / d.n;
  const int64_t j = r - i * d.n;
  int64_t oa, ob;
  batch_offsets(d, b, oa, ob);
  const float2* A = reloc<const float2>(d.A, e.rel_a, arena) + oa;
  const float2* B = reloc<const float2>(d.B, e.rel_b, arena) + ob;
  float2* C = reloc<float2>(d.C, e.rel_c, arena);
  float cr = 0.f, ci = 0.f, crx = 0.f, cix = 0.f;
  if (d.kA || d.kB) {  // in-place leaf operands (tables, per-chunk base offsets)
    A += (e.slot_a >= 0 ? bases[e.slot_a] : 0) + (d.rowA ? d.rowA[i] : i * row_stride(d));
    B += (e.slot_b >= 0 ? bases[e.slot_b] : 0) + (d.rowB ? d.rowB[j] : j * row_stride(d));
    cdot_tables<SPLIT>(A, d.kA, B, d.kB, d.k, cr, ci, crx, cix);
  } else {
    cdot_serial<SPLIT>(A + i * row_stride(d), B + j * row_stride(d), d.k, cr, ci, crx, cix);
  }
  const int64_t c = b * mn + (d.offM ? d.offM[i] + d.offN[j] : r);
  if constexpr (SPLIT)
    C[c] = make_float2(cr + crx, ci + cix);
  else
    C[c] = make_float2(cr, ci);
}

// Work item gt of a level's grouped leaf gathers: one output element.
__device__ __forceinline__ void gather_item(const GroupGather* __restrict__ g, const int64_t* __restrict__ prefix,
                                            int n, int64_t gt, char* arena, const int64_t* bases) {
  const int s = find_item(prefix, n, gt);
  const GroupGather& e = g[s];
  int64_t rest = gt - prefix[s];
  int64_t off = e.base_slot >= 0 ? bases[e.base_slot] : 0;
  for (int j = e.rank - 1; j >= 0; --j) {
    const int64_t x = e.ext[j];
    const int64_t q = rest / x;
    off += (rest - q * x) * e.in_stride[j];
    rest = q;
  }
  reinterpret_cast<float2*>(arena + e.out_off)[gt - prefix[s]] = e.in[off];
}

// the run holding work item gt (runs in launch order, a few dozen at most)
__device__ __forceinline__ int find_run(const GroupRun* runs, int n_runs, int64_t gt) {
  int r = 0;
  while (r + 1 < n_runs && runs[r + 1].first <= gt) ++r;
  return r;
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void group_small_gemm(const GroupGemm* __restrict__ g, const int64_t* __restrict__ prefix,
                                                        int n, int64_t total, char* arena, const int64_t* bases) {
  for (int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; gt < total;
       gt += static_cast<int64_t>(gridDim.x) * blockDim.x)
    small_gemm_item<SPLIT>(g, prefix, n, gt, arena, bases);
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void group_small_gemm_runs(const GroupRun* __restrict__ runs, int n_runs,
                                                             int64_t total) {
  for (int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; gt < total;
       gt += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const GroupRun& q = runs[find_run(runs, n_runs, gt)];
    small_gemm_item<SPLIT>(static_cast<const GroupGemm*>(q.table), q.prefix, q.n, gt - q.first, q.arena, q.bases);
  }
}

__global__ __launch_bounds__(256) void group_gather(const GroupGather* __restrict__ g, const int64_t* __restrict__ prefix,
                                                    int n, int64_t total, char* arena, const int64_t* bases) {
  for (int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; gt < total;
       gt += static_cast<int64_t>(gridDim.x) * blockDim.x)
    gather_item(g, prefix, n, gt, arena, bases);
}

__global__ __launch_bounds__(256) void group_gather_runs(const GroupRun* __restrict__ runs, int n_runs, int64_t total) {
  for (int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; gt < total;
       gt += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const GroupRun& q = runs[find_run(runs, n_runs, gt)];
    gather_item(static_cast<const GroupGather*>(q.table), q.prefix, q.n, gt - q.first, q.arena, q.bases);
  }
}

int64_t grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g < 1) g = 1;
  return g > 1048576 ? 1048576 : g;
}

}  // namespace

hipError_t launch_group_gemm(const GroupGemm* table, const int64_t* prefix, int n, int64_t total, char* arena,
                             const int64_t* bases, Prec prec, hipStream_t s) {
  if (n <= 0 || total <= 0) return hipSuccess;
  if (prec == Prec::BF16X3)
    hipLaunchKernelGGL(group_small_gemm<true>, dim3(grid_for(total)), dim3(256), 0, s, table, prefix, n, total, arena,
                       bases);
  else
    hipLaunchKernelGGL(group_small_gemm<false>, dim3(grid_for(total)), dim3(256), 0, s, table, prefix, n, total, arena,
                       bases);
  return hipGetLastError();
}

hipError_t launch_group_gather(const GroupGather* table, const int64_t* prefix, int n, int64_t total, char* arena,
                               const int64_t* bases, hipStream_t s) {
  if (n <= 0 || total <= 0) return hipSuccess;
  hipLaunchKernelGGL(group_gather, dim3(grid_for(total)), dim3(256), 0, s, table, prefix, n, total, arena, bases);
  return hipGetLastError();
}

hipError_t launch_group_gemm_runs(const GroupRun* runs, int n_runs, int64_t total, Prec prec, hipStream_t s) {
  if (n_runs <= 0 || total <= 0) return hipSuccess;
  if (prec == Prec::BF16X3)
    hipLaunchKernelGGL(group_small_gemm_runs<true>, dim3(grid_for(total)), dim3(256), 0, s, runs, n_runs, total);
  else
    hipLaunchKernelGGL(group_small_gemm_runs<false>, dim3(grid_for(total)), dim3(256), 0, s, runs, n_runs, total);
  return hipGetLastError();
}

hipError_t launch_group_gather_runs(const GroupRun* runs, int n_runs, int64_t total, hipStream_t s) {
  if (n_runs <= 0 || total <= 0) return hipSuccess;
  hipLaunchKernelGGL(group_gather_runs, dim3(grid_for(total)), dim3(256), 0, s, runs, n_runs, total);
  return hipGetLastError();
}

}  // namespace tnc
