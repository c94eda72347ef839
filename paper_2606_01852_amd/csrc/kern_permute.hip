// Operand permutation kernels (complex64 bit copies).
//
// A step's operand must be stored [retained || reduced] (paper Sec. IV-A);
// leaves whose stored order differs, and leaves of a slice batch, are
// rewritten once before the step that reads them.  The tiled kernel moves
// one tile per iteration through LDS: it reads a tile whose innermost modes
// are the input's innermost ones (contiguous runs) and writes it back with
// the output's innermost modes innermost (contiguous runs), so both sides of
// HBM traffic are coalesced.  All index arithmetic is precomputed on the
// host into small tables; the kernel only adds offsets.
//
// Loads and stores are non-temporal: every element is read once and written
// once, and the output (gigabytes for the large operands) is consumed by a
// later launch, so neither side is kept in the caches.  Launches use many
// short-lived workgroups (each loops over a few tiles), so the tiles in
// flight at any moment are a narrow window of the tensor.  On pair30's
// 2^30-element operand both together moved the kernel from 5.1 to 5.7 TB/s
// (a plain copy kernel built the same way: 6.2 TB/s).
#include <mutex>
#include <type_traits>

#include "bf16_split.hpp"
#include "kernels.hpp"

// Table area of the permutes that allocate nothing: the index tables of
// such a call are copied here instead of into memory the library allocates.
// Each GPU holds its own copy of the array at its own address; host code
// uses only the address looked up per device below, never this name (in
// host code it does not denote device memory).
static __device__ __align__(256) unsigned char scratch[tnc::kStaticPermuteTableBytes];

namespace tnc {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_table_mu;
void* g_table_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_table_area(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_table_mu);
  if (!g_table_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_table_ptr[device] = p;
  }
  *out = g_table_ptr[device];
  return hipSuccess;
}

namespace {

constexpr int kPermThreads = 256;

typedef float f2v __attribute__((ext_vector_type(2)));

// Output element o of a permutation: complex64, or its split into the
// planes of a split-precision GEMM operand (PermuteDesc::planes).
template <int PLANES>
__device__ __forceinline__ void put_out(f2v* __restrict__ out, int64_t o, f2v v, const PermuteDesc& d,
                                        double inv_pk) {
  if constexpr (PLANES == 0)
    __builtin_nontemporal_store(v, out + o);
  else if constexpr (PLANES == 1)
    put_planes_a(reinterpret_cast<uint32_t*>(out), o, v.x, v.y);
  else if constexpr (PLANES == 2)
    put_planes_b(reinterpret_cast<uint32_t*>(out), o, d.pk, inv_pk, v.x, v.y);
  else
    put_planes_3m(reinterpret_cast<uint32_t*>(out), o, d.pk, inv_pk, d.pplane, v.x, v.y);
}

template <int EPT, int PLANES>
__global__ __launch_bounds__(kPermThreads) void permute_tiled(PermuteDesc d) {
  extern __shared__ f2v lds[];
  const f2v* __restrict__ in = reinterpret_cast<const f2v*>(d.in);
  f2v* __restrict__ out = reinterpret_cast<f2v*>(d.out);
  const int t = threadIdx.x;
  int32_t in_off[EPT], slot_r[EPT], out_off[EPT], slot_w[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int idx = e * kPermThreads + t;
    const bool ok = idx < d.T;
    in_off[e] = ok ? d.tile_in[idx] : -1;
    slot_r[e] = ok ? d.tile_slot_r[idx] : 0;
    out_off[e] = ok ? d.tile_out[idx] : -1;
    slot_w[e] = ok ? d.tile_slot_w[idx] : 0;
  }
  const int64_t base = d.base + (d.base_dev ? d.base_dev[0] : 0);
  const uint32_t L = static_cast<uint32_t>(d.L);
  const double inv_pk = PLANES >= 2 ? 1.0 / static_cast<double>(d.pk) : 0.0;
  int64_t tile = blockIdx.x;
  if (tile >= d.n_tiles) return;
  f2v v[EPT];
  auto load = [&](int64_t tl) {
    const uint32_t hi = static_cast<uint32_t>(tl / L);
    const uint32_t lo = static_cast<uint32_t>(tl - static_cast<int64_t>(hi) * L);
    const int64_t ib = base + d.lo_tab[2 * lo] + d.hi_tab[2 * hi];
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (in_off[e] >= 0) v[e] = __builtin_nontemporal_load(in + ib + in_off[e]);
  };
  load(tile);
  for (; tile < d.n_tiles; tile += gridDim.x) {
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (in_off[e] >= 0) lds[slot_r[e]] = v[e];
    __syncthreads();
    const int64_t next = tile + gridDim.x;
    const uint32_t hi = static_cast<uint32_t>(tile / L);
    const uint32_t lo = static_cast<uint32_t>(tile - static_cast<int64_t>(hi) * L);
    const int64_t ob = d.lo_tab[2 * lo + 1] + d.hi_tab[2 * hi + 1];
    if (next < d.n_tiles) load(next);
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (out_off[e] >= 0) put_out<PLANES>(out, ob + out_off[e], lds[slot_w[e]], d, inv_pk);
    __syncthreads();
  }
}

// The same tile moved as 16-byte pairs (PermuteDesc::pairs): thread slot p
// carries read-order elements 2p, 2p + 1 (adjacent in the input) and
// write-order elements 2p, 2p + 1 (adjacent in the output), one 16-byte
// load and one 16-byte store each, through the same LDS slots.
typedef float f4v __attribute__((ext_vector_type(4)));

template <int PPT, int PLANES>
__global__ __launch_bounds__(kPermThreads) void permute_pairs(PermuteDesc d) {
  extern __shared__ f2v lds[];
  const f2v* __restrict__ in = reinterpret_cast<const f2v*>(d.in);
  f2v* __restrict__ out = reinterpret_cast<f2v*>(d.out);
  const int t = threadIdx.x;
  const int P = d.T >> 1;
  int32_t in_off[PPT], sr0[PPT], sr1[PPT], out_off[PPT], sw0[PPT], sw1[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int p = e * kPermThreads + t;
    const bool ok = p < P;
    in_off[e] = ok ? d.tile_in[2 * p] : -1;
    sr0[e] = ok ? d.tile_slot_r[2 * p] : 0;
    sr1[e] = ok ? d.tile_slot_r[2 * p + 1] : 0;
    out_off[e] = ok ? d.tile_out[2 * p] : -1;
    sw0[e] = ok ? d.tile_slot_w[2 * p] : 0;
    sw1[e] = ok ? d.tile_slot_w[2 * p + 1] : 0;
  }
  const int64_t base = d.base;
  const uint32_t L = static_cast<uint32_t>(d.L);
  const double inv_pk = PLANES >= 2 ? 1.0 / static_cast<double>(d.pk) : 0.0;
  int64_t tile = blockIdx.x;
  if (tile >= d.n_tiles) return;
  f4v v[PPT];
  auto load = [&](int64_t tl) {
    const uint32_t hi = static_cast<uint32_t>(tl / L);
    const uint32_t lo = static_cast<uint32_t>(tl - static_cast<int64_t>(hi) * L);
    const int64_t ib = base + d.lo_tab[2 * lo] + d.hi_tab[2 * hi];
#pragma unroll
    for (int e = 0; e < PPT; ++e)
      if (in_off[e] >= 0) v[e] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(in + ib + in_off[e]));
  };
  load(tile);
  for (; tile < d.n_tiles; tile += gridDim.x) {
#pragma unroll
    for (int e = 0; e < PPT; ++e)
      if (in_off[e] >= 0) {
        lds[sr0[e]] = v[e].xy;
        lds[sr1[e]] = v[e].zw;
      }
    __syncthreads();
    const int64_t next = tile + gridDim.x;
    const uint32_t hi = static_cast<uint32_t>(tile / L);
    const uint32_t lo = static_cast<uint32_t>(tile - static_cast<int64_t>(hi) * L);
    const int64_t ob = d.lo_tab[2 * lo + 1] + d.hi_tab[2 * hi + 1];
    if (next < d.n_tiles) load(next);
#pragma unroll
    for (int e = 0; e < PPT; ++e)
      if (out_off[e] >= 0) {
        const f2v a = lds[sw0[e]], b = lds[sw1[e]];
        const int64_t o = ob + out_off[e];
        if constexpr (PLANES == 0)
          __builtin_nontemporal_store(f4v{a.x, a.y, b.x, b.y}, reinterpret_cast<f4v*>(out + o));
        else if constexpr (PLANES == 1)
          put_planes_a2(reinterpret_cast<uint32_t*>(out), o, a.x, a.y, b.x, b.y);
        else if constexpr (PLANES == 2)
          put_planes_b2(reinterpret_cast<uint32_t*>(out), o, d.pk, inv_pk, a.x, a.y, b.x, b.y);
        else
          put_planes_3m2(reinterpret_cast<uint32_t*>(out), o, d.pk, inv_pk, d.pplane, a.x, a.y, b.x, b.y);
      }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void gather_plain(GatherDesc d) {
  const int64_t base = d.base + (d.base_dev ? d.base_dev[0] : 0);
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < d.total;
       w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int64_t rest = w, off = base;
    for (int j = d.rank - 1; j >= 0; --j) {
      const int64_t e = d.ext[j];
      const int64_t q = rest / e;
      off += (rest - q * e) * d.in_stride[j];
      rest = q;
    }
    d.out[w] = d.in[off];
  }
}

}  // namespace

hipError_t launch_permute(const PermuteDesc& d, hipStream_t s) {
  if (d.n_tiles <= 0) return hipSuccess;
  // 16 elements per thread for every tile of up to 4096 elements: measured
  // faster than the smallest fitting count (8 for pair30's 2048-element
  // tiles: 5.69 vs 5.77 TB/s), which runs twice the waves per CU
  int ept = 1;
  while (ept * kPermThreads < d.T) ept *= 2;
  if (d.n_tiles >= 1024 && ept < 16) ept = 16;
  const size_t lds = static_cast<size_t>(d.slots) * sizeof(float2);
  // many short-lived workgroups of about 8192 elements (64 KiB) each: a
  // few tiles per workgroup, so each loads its next tile while it stores
  // the current one.  Measured: 131072 workgroups best among 8192 .. one
  // per tile on pair30's 2^30-element operand (4096-element tiles); 1024-
  // element tiles of 2^28 elements 0.94 -> 0.85 ms at 32768 instead of
  // 131072, pair_batch's 64 operand permutes 0.164 -> 0.125 ms.  At least
  // 1024 workgroups (or one per tile) so that small tensors stay spread
  // over the chip.
  int64_t grid = d.n_tiles * d.T / 8192;
  if (grid < 1024) grid = 1024;
  if (grid > d.n_tiles) grid = d.n_tiles;
  if (grid > 131072) grid = 131072;
  // 16-byte pairs where the tables allow them and the base keeps them
  // aligned (standalone repeats of pair30's 2^30-element permutation:
  // 5.77 -> 5.92 TB/s; pair_batch's 64 operand permutes: 0.198 -> 0.165
  // ms); pairs per thread follow the element rule (8 pairs where it takes
  // 16 elements)
  const bool aligned = (reinterpret_cast<uintptr_t>(d.in) | reinterpret_cast<uintptr_t>(d.out)) % 16 == 0;
  if (d.planes < 0 || d.planes > 3 || (d.planes && (d.pk <= 0 || d.pk % (d.planes == 3 ? 32 : 16) != 0)) ||
      (d.planes == 3 && d.pplane <= 0))
    return hipErrorInvalidValue;
  auto launch = [&](auto plane_tag) -> hipError_t {
    constexpr int PL = decltype(plane_tag)::value;
    if (d.pairs && !d.base_dev && d.base % 2 == 0 && aligned && ept >= 2) {
      switch (ept / 2) {
#define TNC_PAIR_CASE(E) \
  case E: hipLaunchKernelGGL((permute_pairs<E, PL>), dim3(grid), dim3(kPermThreads), lds, s, d); return hipGetLastError();
        TNC_PAIR_CASE(1)
        TNC_PAIR_CASE(2)
        TNC_PAIR_CASE(4)
        TNC_PAIR_CASE(8)
#undef TNC_PAIR_CASE
        default: break;
      }
    }
    switch (ept) {
#define TNC_PERM_CASE(E) \
  case E: hipLaunchKernelGGL((permute_tiled<E, PL>), dim3(grid), dim3(kPermThreads), lds, s, d); break;
      TNC_PERM_CASE(1)
      TNC_PERM_CASE(2)
      TNC_PERM_CASE(4)
      TNC_PERM_CASE(8)
      TNC_PERM_CASE(16)
#undef TNC_PERM_CASE
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  if (d.planes == 1) return launch(std::integral_constant<int, 1>{});
  if (d.planes == 2) return launch(std::integral_constant<int, 2>{});
  if (d.planes == 3) return launch(std::integral_constant<int, 3>{});
  return launch(std::integral_constant<int, 0>{});
}

hipError_t launch_gather(const GatherDesc& d, hipStream_t s) {
  if (d.total <= 0) return hipSuccess;
  int64_t grid = (d.total + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(gather_plain, dim3(grid), dim3(256), 0, s, d);
  return hipGetLastError();
}

}  // namespace tnc
