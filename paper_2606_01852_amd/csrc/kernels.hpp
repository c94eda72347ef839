// Internal kernel interface: descriptors built by the host planner and the
// launchers that run them.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tnc {

constexpr int kMaxBatchDims = 24;

// Batched complex GEMM  C[b, i, j] = sum_l A[b, i, l] * B[b, j, l].
// A, B are K-contiguous ([.. | M | K] and [.. | N | K] storage, row stride
// ldk, which is k when ldk is 0).  The batch index b (0 <= b < h) is
// row-major over nbd batch dims; the operands' offsets are
// sum_d digit_d * bs{A,B}[d] (0 = broadcast), C's is b * m * n.  Within one
// batch entry C is natural row-major [m, n] when offM is null, else element
// (i, j) sits at offM[i] + offN[j].  A split of the K range into S parts is
// expressed as one more (innermost) batch dim of extent S with strides
// k / S, k = k / S and ldk = the full row length; the S partial products
// are then summed by launch_splitk_reduce.
struct GemmDesc {
  const float2* A;
  const float2* B;
  float2* C;
  int64_t m, n, k, h;
  int32_t nbd;
  int32_t pow2;                    // every batch extent a power of two
  int32_t bext[kMaxBatchDims];
  int32_t bshift[kMaxBatchDims];   // log2(bext) when pow2
  int64_t bsA[kMaxBatchDims];
  int64_t bsB[kMaxBatchDims];
  const int64_t* offM;
  const int64_t* offN;
  int64_t ldk;
  // Operands read in place through tables (leaves whose sliced labels are
  // fixed per chunk, consumed by the one-thread-per-output kernels only):
  // element (b, i, l) of A is A[batch offset + *baseA + rowA[i] + kA[l]]
  // (B likewise); null tables: i * ldk + l, null base: 0.
  const int64_t* rowA;
  const int64_t* kA;
  const int64_t* baseA;
  const int64_t* rowB;
  const int64_t* kB;
  const int64_t* baseB;
};

__host__ __device__ inline int64_t row_stride(const GemmDesc& d) { return d.ldk ? d.ldk : d.k; }

enum class Form : int { M4 = 0, M3 = 1 };
enum class Prec : int { C64 = 0, BF16X3 = 1 };
enum class GemmKernel : int { MFMA = 0, SMALL = 1, DOT = 2 };

// Kernel choice for one step's shape (shared by the planner and the
// stand-alone GEMM entry point).
//  * MFMA for shapes that fill its 64 x 32 wave tiles, and for skinny shapes
//    (m >= 16, n >= 8) with enough work (2^22 complex MACs) that running
//    MFMA on padded tiles still beats one thread per output;
//  * DOT (one wave64 per output) for long reductions with few outputs;
//  * SMALL (one thread per output) for the rest: tiny steps.
inline GemmKernel choose_gemm_kernel(int64_t h, int64_t m, int64_t n, int64_t k) {
  const int64_t tiles = ((m + 127) / 128) * ((n + 63) / 64) * h;
  const int64_t work = h * m * n * k;  // complex MACs
  if (k >= 16 && tiles < (int64_t{1} << 24)) {
    // below 2^22 MACs a short-K step covers a few MFMA workgroups that each
    // loop over K alone; one thread per output finishes it sooner (64 x 64 x
    // 64: 11.7 vs 14.9 us) and joins its tree level's grouped launch
    if (m >= 64 && n >= 32 && (work >= (int64_t{1} << 22) || k > 128)) return GemmKernel::MFMA;
    if (m >= 16 && n >= 8 && work >= (int64_t{1} << 22)) return GemmKernel::MFMA;
  }
  if (k >= 256 && m * n <= 64 && (h * m * n + 3) / 4 < 0x7FFFFF) return GemmKernel::DOT;
  return GemmKernel::SMALL;
}

// Tiled gather-permute of complex64: out (contiguous) gets, for every tile
// t < n_tiles and element e < T of the tile,
//   out[tile_out_base(t) + tile_out[e]] = in[base + tile_in_base(t) + tile_in[e']]
// where the per-tile bases come from two host-built tables (outer tile index
// split row-major into hi * L + lo) and the in-tile offsets and LDS slots
// from per-element tables (read order r and write order w).
struct PermuteDesc {
  const float2* in;
  float2* out;
  const int32_t* tile_in;      // [T] input offset of read-order element r
  const int32_t* tile_slot_r;  // [T] LDS slot of read-order element r
  const int32_t* tile_out;     // [T] output offset of write-order element w
  const int32_t* tile_slot_w;  // [T] LDS slot of write-order element w
  const int64_t* lo_tab;       // [L * 2] (in, out) offsets of the low outer digits
  const int64_t* hi_tab;       // [Hn * 2] (in, out) offsets of the high outer digits
  int64_t n_tiles;
  int32_t L;
  int32_t T;
  int32_t slots;               // LDS slots used (>= T, padding included)
  int64_t base;                // constant input offset
  const int64_t* base_dev;     // optional extra input offset read on device
  int32_t pairs;               // the tables allow 16-byte pairs (PermuteHost::pairs)
  // 0: write complex64 to out; 1 / 2: write the split planes of a
  // split-precision GEMM's A / B' operand (out = the planes, rows of pk
  // complex, pk a multiple of 16); 3: the r, i and s planes of a 3M-form
  // operand (rows of pk complex, pk a multiple of 32, the i and s planes
  // pplane uint32 after the r planes)
  int32_t planes;
  int64_t pk;
  int64_t pplane;
};

// Plain gather: out[w] = in[base + sum_d digit_d(w) * in_stride[d]] over
// row-major output dims (any shape; used for small tensors).
constexpr int kMaxRank = 64;
struct GatherDesc {
  const float2* in;
  float2* out;
  int64_t total;
  int32_t rank;
  int64_t ext[kMaxRank];
  int64_t in_stride[kMaxRank];
  int64_t base;
  const int64_t* base_dev;
};

// MFMA tile variants: variant v uses workgroups of WM x WN wave64, each
// wave owning 64 x 32 complex of C (gemm_variant_tile gives the block tile).
constexpr int kGemmVariants = 7;
void gemm_variant_tile(int variant, int* bm, int* bnc);
// Allow every MFMA kernel instance its LDS on the current device (best
// effort; launches do it lazily as well).
void prepare_gemm_kernels();
hipError_t launch_gemm(const GemmDesc& d, GemmKernel kind, int variant, Form form, Prec prec, hipStream_t s);
// Grouped MFMA launch: several GEMMs (any shapes, pointers, batch strides
// and store tables) that share one tile variant, precision and form, run by
// one persistent launch whose workgroups loop over the tiles of all of them.
// Every tile is computed exactly as the single-GEMM kernel of that variant
// computes it, so each result is bitwise the same as a launch of its own.
// Entries need even k and row stride (16-byte operand loads).  Grouped
// forms exist only where the persistent tile loop fits the registers
// without spilling (grouped_variant_ok: every 4M variant, 3M but 3, split
// precision's 0 and 4-6); other launches fail with hipErrorInvalidValue.
struct GroupedEntry {
  GemmDesc d;
  int64_t tiles_m, tiles_n;   // tile grid of one batch entry
  int64_t tile0;              // first tile of this entry in the launch
};
// Fill tiles_m, tiles_n and tile0 of e[0..n) for `variant`; returns the
// launch's total tiles (0 when an entry cannot run grouped: odd k or row
// stride).
int64_t grouped_layout(GroupedEntry* e, int n, int variant);
// `dev` is the device copy of the n entries laid out by grouped_layout.
bool grouped_variant_ok(Form form, Prec prec, int variant);
hipError_t launch_gemm_grouped(const GroupedEntry* dev, int n, int64_t total, int variant, Form form, Prec prec,
                               hipStream_t s);
hipError_t launch_gemm_valu(const GemmDesc& d, GemmKernel kind, Prec prec, hipStream_t s);
// Split-bf16x3 on operands split once into bf16 planes (large steps of one
// batch entry, h == 1, no operand tables): the launch splits A and B into
// `planes` (presplit_plane_bytes(m, n, k) bytes of device memory, 256-byte
// aligned) and runs the 256 x 128 wide-wave tile on them with direct
// global -> LDS staging.  Bitwise the result of the wide-wave variant (3).
constexpr int64_t kPresplitBM = 256, kPresplitBNC = 128;
inline int64_t presplit_rows_a(int64_t m) { return (m + kPresplitBM - 1) / kPresplitBM * kPresplitBM; }
inline int64_t presplit_rows_b(int64_t n) { return 2 * ((n + kPresplitBNC - 1) / kPresplitBNC * kPresplitBNC); }
inline int64_t presplit_k(int64_t k) { return (k + 15) / 16 * 16; }
inline size_t presplit_plane_bytes(int64_t m, int64_t n, int64_t k) {
  // per row and 16 complex k: 128 bytes (32 bf16 hi, 32 bf16 lo)
  return static_cast<size_t>((presplit_rows_a(m) + presplit_rows_b(n)) * presplit_k(k) * 8);
}
// have_a / have_b: that operand's planes are already written (by the
// permute that produced it) and are not split again.
hipError_t launch_gemm_presplit(const GemmDesc& d, void* planes, bool have_a, bool have_b, hipStream_t s);
// The 3M form on the same kernel: each operand's real parts X_r, X_i and
// X_s = X_r + X_i (float32 sums) are split once into the planes of a real
// GEMM operand (rows of 2 kp real k), the three real products T1 = A_r B_r^T,
// T2 = A_i B_i^T, T3 = A_s B_s^T run as three launches of the pre-split
// kernel into float32 matrices of m x 2 nh, and a last pass forms
// C = (T1 - T2, T3 - T1 - T2) with the step's store.  Bitwise the result
// of the 3M split tiles (same products in the same order per accumulator).
// `buf`: presplit_3m_layout(m, n, k).bytes of device memory, 256-aligned.
struct Presplit3M {
  int64_t mp, np, kp, nh;      // padded rows of A and B, real k pairs, column pairs of T
  int64_t off_b, off_t;        // byte offsets of B's planes and of T1 in the buffer
  int64_t tplane;              // floats from T1 to T2 (and T2 to T3)
  int64_t bytes;
};
inline Presplit3M presplit_3m_layout(int64_t m, int64_t n, int64_t k) {
  auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
  Presplit3M g;
  g.nh = (n + 1) / 2;
  g.mp = presplit_rows_a(m);
  g.np = presplit_rows_b(g.nh);      // real rows of B, padded to the tile's 256
  g.kp = presplit_k((k + 1) / 2);    // real k pairs per row: k padded to 32
  g.off_b = al(3 * g.mp * g.kp * 8);  // per row 2 kp real k, hi and lo: 8 kp bytes
  g.off_t = g.off_b + al(3 * g.np * g.kp * 8);
  g.tplane = m * 2 * g.nh;
  g.bytes = g.off_t + al(3 * g.tplane * 4);
  return g;
}
// have_a / have_b: as for launch_gemm_presplit (rows of k complex, k a
// multiple of 32, written by the permute that produced the operand).
hipError_t launch_gemm_presplit_3m(const GemmDesc& d, void* buf, bool have_a, bool have_b, hipStream_t s);
// Split-K epilogue: C[b, i, j] = sum_{p < S} P[((b * S + p) * m + i) * n + j],
// p ascending, stored at b * m * n + (offM ? offM[i] + offN[j] : i * n + j).
hipError_t launch_splitk_reduce(const float2* P, float2* C, int64_t h, int64_t m, int64_t n, int64_t S,
                                const int64_t* offM, const int64_t* offN, hipStream_t s);
// Grouped launches (one per tree level).  Operand pointers flagged rel_*
// hold arena offsets, relocated against the arena base at run time, so the
// tables stay valid for any arena.
struct GroupGemm {
  GemmDesc d;
  int32_t rel_a, rel_b, rel_c, pad;
  int32_t slot_a, slot_b;   // per-chunk base offset of an in-place operand (-1: none)
};
constexpr int kGroupRank = 32;
struct GroupGather {
  const float2* in;     // resident leaf
  int64_t out_off;      // arena offset of the gathered copy
  int32_t rank;
  int32_t base_slot;    // slot of the chunk's base offset (-1: none)
  int64_t ext[kGroupRank];
  int64_t in_stride[kGroupRank];
};
// prefix[i] = first work item of entry i (work items: output elements).
// An in-place operand's base offset comes from bases[slot_a].
hipError_t launch_group_gemm(const GroupGemm* table, const int64_t* prefix, int n, int64_t total, char* arena,
                             const int64_t* bases, Prec prec, hipStream_t s);
hipError_t launch_group_gather(const GroupGather* table, const int64_t* prefix, int n, int64_t total, char* arena,
                               const int64_t* bases, hipStream_t s);
// One run's share of a grouped launch over several runs of one structure
// (a fused serving job): its own device table and prefix sums (those of a
// launch of its own), its arena, its current leaf base offsets, and its
// first work item in the launch.  A launch over runs does per work item
// exactly what the run's own launch does.
struct GroupRun {
  const void* table;        // GroupGemm[] or GroupGather[]
  const int64_t* prefix;
  char* arena;
  const int64_t* bases;
  int64_t first;
  int32_t n;
  int32_t pad;
};
hipError_t launch_group_gemm_runs(const GroupRun* runs, int n_runs, int64_t total, Prec prec, hipStream_t s);
hipError_t launch_group_gather_runs(const GroupRun* runs, int n_runs, int64_t total, hipStream_t s);

hipError_t launch_permute(const PermuteDesc& d, hipStream_t s);
// Fixed device-resident table area for permutes of callers that cannot
// allocate (tnc_permute_noalloc): kStaticPermuteTableBytes per GPU, shared
// by every such call on that GPU.  static_table_area looks its address up
// once per device (the device must be current) and returns it.
constexpr size_t kStaticPermuteTableBytes = size_t{1} << 20;
hipError_t static_table_area(int device, void** out);
hipError_t launch_gather(const GatherDesc& d, hipStream_t s);
// acc[i] += sum_s root[s * R + i] (complex64 in, complex128 out), pairwise
// over s in a fixed tree; hs = number of s.  overwrite: acc[i] = the sum
// (the same bits as adding it to a zeroed accumulator).
hipError_t launch_reduce_fp64(const float2* root, double2* acc, int64_t hs, int64_t R, bool overwrite,
                              hipStream_t s);
// out = sum_i |acc[i]|^2 in FP64 (one value written to *out, device pointer).
hipError_t launch_norm2(const double2* acc, int64_t R, double* out, hipStream_t s);
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s);
// p[i] = a hash of (i, seed) mapped to [-1, 1), i < n floats (autotuner
// stand-in operands).
hipError_t launch_fill_hash(float* p, int64_t n, uint32_t seed, hipStream_t s);
// Calibration: `blocks` workgroups of 256 threads running `iters` rounds of
// 8 FP32 16x16x4 MFMAs per wave (out: blocks * 256 floats, never written in
// practice); a grid-stride 16-byte copy of `bytes` (a multiple of 16).
hipError_t launch_mfma_rate(float* out, int blocks, int iters, hipStream_t s);
hipError_t launch_copy_rate(const void* in, void* out, int64_t bytes, hipStream_t s);
// complex128 -> complex64 conversion (leaf upload).
hipError_t launch_c128_to_c64(const double2* in, float2* out, int64_t n, hipStream_t s);

}  // namespace tnc
