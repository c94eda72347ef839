// Batched complex GEMM on MFMA for gfx950:  C[b,i,j] = sum_l A[b,i,l] B[b,j,l].
//
// Every contraction step of the path is one such GEMM once the operands are
// in [retained || reduced] order (paper Sec. II-B: A_MK x B_KN -> C_MN;
// Sec. IV-A: the canonical operand layout maps directly to a GEMM).  Both
// operands are K-contiguous, so the product is A * B^T per batch entry.
//
// 4M form on FP32 MFMA.  A complex row of A, read as 2k floats
// (ar0, ai0, ar1, ai1, ...), times the real 2k-vector
//   (br0, -bi0, br1, -bi1, ...)  gives Re C,
//   (bi0,  br0, bi1,  br1, ...)  gives Im C,
// so C, viewed as an m x 2n float matrix, is a single real GEMM of
// m x 2n x 2k whose B operand is built in registers from B's interleaved
// values (a lane-dependent select and sign flip).  The MFMA output columns
// then alternate re/im: exactly the interleaved complex64 layout, with no
// de-interleaving anywhere.  8 real FLOPs per complex MAC (the paper's
// counting convention, Sec. II-B).
//
// 3M form: T1 = Ar Br, T2 = Ai Bi, T3 = (Ar+Ai)(Br+Bi), Re = T1 - T2,
// Im = T3 - T1 - T2: three real GEMMs, 6 executed FLOPs per complex MAC.
//
// BF16x3: each float32 plane is split into bf16 hi/lo (round to nearest
// even) while it is staged into LDS; every real product becomes
// a_hi b_hi + (a_hi b_lo + a_lo b_hi) on bf16 MFMA with FP32 accumulation
// (hi and cross terms in separate accumulators; in the wide-wave variant
// and the 3M form, one accumulator per real product).  It composes with
// both forms: 12 bf16 products per complex product in the 4M form, 9 in
// the 3M form (the sum planes Ar+Ai, Br+Bi formed in float32, then split).
// Large single GEMMs split their operands once into bf16 planes in global
// memory instead and stage them straight into LDS (the pre-split section
// below); in the 3M form as three real GEMMs plus a combining pass.
//
// Tiling.  A wave64 owns a 64 x 32 complex tile of C (2x2 MFMA 32x32 blocks
// of the real view, or 2x1 complex blocks in 3M); a workgroup is WM x WN
// waves, so its tile is 64*WM x 32*WN complex.  The split-bf16 256 x 128
// tile instead runs 4x2 waves of 64 x 64 complex each (2x4 blocks).  K advances 16
// complex per stage through double-buffered LDS (rows padded to 144 B: the
// 16-byte fragment reads of 16 lanes hit 16 distinct 4-bank groups).  Each
// lane reads 4 consecutive real k and feeds them to 4 successive MFMAs; the
// K order inside a stage is permuted the same way for A and B.  Interior
// tiles run a copy of the main loop without bounds checks.  Tiles sweep N
// in groups of 8 M-tiles, and workgroups are remapped (the hardware deals
// them round-robin over the 8 XCDs, each with its own L2) so that the tiles
// one XCD runs at once form 8 x 4 blocks: 12 operand panels per 32 tiles
// through its L2.  Where the tile counts allow, the eight XCDs' blocks share
// their 8 M-tiles, so the memory-side cache serves each A panel to all of
// them from one HBM read (split precision on pair30: 316.7 -> 314.5 ms,
// where the chip's power sets its clock; complex64 unchanged).
#include <atomic>
#include <cstring>
#include <type_traits>

#include "bf16_split.hpp"
#include "gemm_common.hpp"

namespace tnc {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));

constexpr int BKC = 16;     // complex k per LDS stage
constexpr int PITCH = 36;   // floats per LDS row (32 data + 4 pad)
constexpr int SPITCH = 40;  // uint16 per LDS row of a bf16 plane (32 data + 8 pad)
constexpr int GROUP_M = 8;

template <int WM, int WN, int PW = 1>
struct Shape {
  static constexpr int BM = 64 * WM;        // rows of C per workgroup
  static constexpr int BNC = 32 * WN * PW;  // complex columns of C per workgroup (PW per wave)
  static constexpr int NT = 64 * WM * WN;
  static constexpr size_t lds_f32 = 2 * (BM + BNC) * PITCH * sizeof(float);
  // bf16 stage: A hi/lo planes of BM rows, B' hi/lo planes of 2*BNC real
  // columns (the 4M real operand, built at staging), two buffers
  static constexpr int BF16_STAGE = (2 * BM + 4 * BNC) * SPITCH;  // uint16 per buffer
  static constexpr size_t lds_bf16 = 2 * BF16_STAGE * sizeof(uint16_t);
};

struct TileCoord {
  int64_t b, row0, col0;
};

// Tile of workgroup index `wg` (already in XCD order) within one GEMM:
// batch entry, then groups of GROUP_M M-tiles swept along N.
template <int BM, int BNC>
__device__ __forceinline__ TileCoord tile_of(int64_t wg, int64_t tiles_m, int64_t tiles_n) {
  const int64_t tpb = tiles_m * tiles_n;
  const int64_t b = wg / tpb;
  const int64_t r = wg - b * tpb;
  const int64_t gw = static_cast<int64_t>(GROUP_M) * tiles_n;
  const int64_t grp = r / gw;
  const int64_t first_m = grp * GROUP_M;
  const int64_t rem_m = tiles_m - first_m;
  const int64_t gsz = rem_m < GROUP_M ? rem_m : GROUP_M;
  const int64_t rr = r - grp * gw;
  TileCoord tc;
  tc.b = b;
  tc.row0 = (first_m + rr % gsz) * BM;
  tc.col0 = (rr / gsz) * BNC;
  return tc;
}

template <int BM, int BNC>
__device__ __forceinline__ TileCoord map_tile(int64_t tiles_m, int64_t tiles_n, int64_t total) {
  int64_t wg = blockIdx.x;
  const int64_t per = total >> 3;
  if (wg < (per << 3)) wg = (wg & 7) * per + (wg >> 3);
  return tile_of<BM, BNC>(wg, tiles_m, tiles_n);
}

// The same 8 x 4 blocks of tiles per XCD, but the eight XCDs work on the
// same eight M-tiles at once (XCD x takes N-tiles x, x + 8, ...): the A
// panels every XCD reads from its own L2 are then shared in the memory-side
// cache, so HBM serves each once instead of once per XCD.  Needs whole
// groups of 64 tiles (tiles_n a multiple of 8, GROUP_M M-tiles per group);
// other shapes keep map_tile's order.
template <int BM, int BNC>
__device__ __forceinline__ TileCoord map_tile_shared(int64_t tiles_m, int64_t tiles_n, int64_t total) {
  const int64_t wg = blockIdx.x;
  if (tiles_n % 8 != 0 || tiles_m % GROUP_M != 0) return map_tile<BM, BNC>(tiles_m, tiles_n, total);
  const int64_t g = wg >> 3, x = wg & 7;
  return tile_of<BM, BNC>(64 * (g >> 3) + 8 * x + (g & 7), tiles_m, tiles_n);
}

// Global -> register staging of one K stage (VW complex per load).  With
// SWZ the rows are dealt to the 8-lane groups in a permuted order within
// each block of 8 rows, so that the two groups of a 16-lane 8-byte LDS store
// cycle hit disjoint banks (rows 80 bytes apart: A rows 4 apart, B' rows 4
// apart = complex columns 2 apart); the data layout itself is unchanged.
template <int WM, int WN, int VW, bool SWZ = false, int PW = 1>
struct Stage {
  using S = Shape<WM, WN, PW>;
  static constexpr int PER_ROW = BKC / VW;
  __device__ __forceinline__ static int row_a(int idx) {
    const int g = idx / PER_ROW;
    if constexpr (SWZ && VW == 2) {
      constexpr int p[8] = {0, 4, 1, 5, 2, 6, 3, 7};
      return (g & ~7) | p[g & 7];
    }
    return g;
  }
  __device__ __forceinline__ static int row_b(int idx) {
    const int g = idx / PER_ROW;
    if constexpr (SWZ && VW == 2) {
      constexpr int p[8] = {0, 2, 1, 3, 4, 6, 5, 7};
      return (g & ~7) | p[g & 7];
    }
    return g;
  }
  static constexpr int A_LOADS = S::BM * PER_ROW / S::NT;
  static constexpr int B_LOADS = S::BNC * PER_ROW / S::NT;
  static_assert(A_LOADS >= 1 && A_LOADS * S::NT == S::BM * PER_ROW, "A staging must tile evenly");
  static_assert(B_LOADS >= 1 && B_LOADS * S::NT == S::BNC * PER_ROW, "B staging must tile evenly");
  f4 a[A_LOADS];
  f4 b[B_LOADS];

  template <bool CHECK>
  __device__ __forceinline__ static f4 fetch(const float2* __restrict__ X, int64_t gr, int64_t gk, int64_t rows,
                                             int64_t k, int64_t ld) {
    f4 v = {0.f, 0.f, 0.f, 0.f};
    if (!CHECK || (gr < rows && gk < k)) {
      const float2* p = X + gr * ld + gk;
      if constexpr (VW == 2) {
        v = *reinterpret_cast<const f4*>(p);
      } else {
        const float2 x = *p;
        v.x = x.x;
        v.y = x.y;
      }
    }
    return v;
  }

  template <bool CHECK>
  __device__ __forceinline__ void load(const float2* __restrict__ A, const float2* __restrict__ B, int64_t m,
                                       int64_t n, int64_t k, int64_t ld, int64_t row0, int64_t col0, int64_t kk,
                                       int tid) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int idx = tid + S::NT * i;
      a[i] = fetch<CHECK>(A, row0 + row_a(idx), kk + (idx % PER_ROW) * VW, m, k, ld);
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int idx = tid + S::NT * i;
      b[i] = fetch<CHECK>(B, col0 + row_b(idx), kk + (idx % PER_ROW) * VW, n, k, ld);
    }
  }

  __device__ __forceinline__ static void put_f32(float* base, int row, int idx, const f4& v) {
    float* p = base + row * PITCH + 2 * (idx % PER_ROW) * VW;
    if constexpr (VW == 2) {
      *reinterpret_cast<f4*>(p) = v;
    } else {
      p[0] = v.x;
      p[1] = v.y;
    }
  }

  __device__ __forceinline__ void store_f32(float* As, float* Bs, int tid) const {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) put_f32(As, row_a(tid + S::NT * i), tid + S::NT * i, a[i]);
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) put_f32(Bs, row_b(tid + S::NT * i), tid + S::NT * i, b[i]);
  }

  // bf16 planes: the hi and lo halves of every float go to separate planes
  // (hardware round-to-nearest-even conversion of two floats at a time,
  // packed [first | second << 16]; lo = rne(x - hi), x - hi exact in
  // float32).
  __device__ __forceinline__ static void split2(float x, float y, uint32_t& hi, uint32_t& lo) {
    bf16_split2(x, y, hi, lo);
  }

  // A: the staged floats in place (real k index = 2 * complex k + re/im).
  __device__ __forceinline__ static void put_split(uint16_t* hi, uint16_t* lo, int idx, const f4& v) {
    const int pos = row_a(idx) * SPITCH + 2 * (idx % PER_ROW) * VW;
    uint32_t h01, l01;
    split2(v.x, v.y, h01, l01);
    if constexpr (VW == 2) {
      uint32_t h23, l23;
      split2(v.z, v.w, h23, l23);
      *reinterpret_cast<uint2*>(hi + pos) = make_uint2(h01, h23);
      *reinterpret_cast<uint2*>(lo + pos) = make_uint2(l01, l23);
    } else {
      *reinterpret_cast<uint32_t*>(hi + pos) = h01;
      *reinterpret_cast<uint32_t*>(lo + pos) = l01;
    }
  }

  // B: complex column c becomes the real columns 2c = (br, -bi, ...) and
  // 2c + 1 = (bi, br, ...) of the 4M operand; negating a bf16 flips its
  // sign bit (which commutes with the split), swapping re/im rotates the
  // packed pair by 16 bits.
  __device__ __forceinline__ static void put_split_b(uint16_t* hi, uint16_t* lo, int idx, const f4& v) {
    const int c = row_b(idx);
    const int pos0 = (2 * c) * SPITCH + 2 * (idx % PER_ROW) * VW;
    const int pos1 = pos0 + SPITCH;
    constexpr uint32_t NEG_IM = 0x80000000u;
    auto swap = [](uint32_t w) { return (w >> 16) | (w << 16); };
    uint32_t h01, l01;
    split2(v.x, v.y, h01, l01);
    if constexpr (VW == 2) {
      uint32_t h23, l23;
      split2(v.z, v.w, h23, l23);
      *reinterpret_cast<uint2*>(hi + pos0) = make_uint2(h01 ^ NEG_IM, h23 ^ NEG_IM);
      *reinterpret_cast<uint2*>(lo + pos0) = make_uint2(l01 ^ NEG_IM, l23 ^ NEG_IM);
      *reinterpret_cast<uint2*>(hi + pos1) = make_uint2(swap(h01), swap(h23));
      *reinterpret_cast<uint2*>(lo + pos1) = make_uint2(swap(l01), swap(l23));
    } else {
      *reinterpret_cast<uint32_t*>(hi + pos0) = h01 ^ NEG_IM;
      *reinterpret_cast<uint32_t*>(lo + pos0) = l01 ^ NEG_IM;
      *reinterpret_cast<uint32_t*>(hi + pos1) = swap(h01);
      *reinterpret_cast<uint32_t*>(lo + pos1) = swap(l01);
    }
  }

  __device__ __forceinline__ void store_split(uint16_t* Ah, uint16_t* Al, uint16_t* Bh, uint16_t* Bl,
                                              int tid) const {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) put_split(Ah, Al, tid + S::NT * i, a[i]);
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) put_split_b(Bh, Bl, tid + S::NT * i, b[i]);
  }
};

// Output offsets within one batch entry of C, in complex elements: a row's
// (offM[row], or row * n) plus a column's (offN[col], or col); -1 marks a
// row or column outside C.  Permuted-store epilogues read them into
// registers before issuing any store: C and the store tables are different
// arrays, but the compiler cannot know it, so a table read between two
// stores would wait for each read in turn.  (Row-major stores compute their
// addresses inline: that keeps the main loop's register allocation, and so
// its schedule, as it is without tables.)
__device__ __forceinline__ int64_t col_offset(const GemmDesc& d, bool perm, int64_t col) {
  return col < d.n ? (perm ? d.offN[col] : col) : -1;
}

// Rows 8*(v>>2) + 4*h + (v&3) of a 32-row MFMA block starting at row0, for
// v = v0 .. v0+7 (the accumulator layout of a 32x32 MFMA).
__device__ __forceinline__ void row_offsets8(const GemmDesc& d, bool perm, int64_t row0, int h, int v0,
                                             int64_t (&o)[8]) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int v = v0 + u;
    const int64_t row = row0 + 8 * (v >> 2) + 4 * h + (v & 3);
    o[u] = row < d.m ? (perm ? d.offM[row] : row * d.n) : -1;
  }
}

// Permuted store of a wave's 64 x 32 complex block held in the 4M layout
// (MFMA 32x32 accumulators over real columns: even lanes hold the real and
// odd lanes the imaginary part of one complex column, for rows v and v+1 of
// each register pair).  One lane swap lets the even lane store row v's
// complex value and the odd lane row v+1's, as 8-byte stores (half the
// store instructions of a 4-byte store per part); each lane reads only the
// row offsets of the rows it stores.  The swap runs in both lanes of a pair
// whatever their row bounds (the column bound is shared by the pair).
// val(i, j, v) is the lane's accumulated value of MFMA block (i, j), entry v.
template <int PW = 1, class Val>
__device__ __forceinline__ void store_perm_pairs(const GemmDesc& d, const TileCoord& tc, int wm, int wn, int lane,
                                                 Val val) {
  constexpr int NJ = 2 * PW;  // 32-real-column blocks per wave
  const int h = lane >> 5, l32 = lane & 31;
  const bool odd = l32 & 1;
  float2* Cz = d.C + tc.b * d.m * d.n;
  int64_t co[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) co[j] = col_offset(d, true, (tc.col0 * 2 + wn * 64 * PW + j * 32 + l32) >> 1);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v0 = 0; v0 < 16; v0 += 8) {
      // this lane stores rows v = v0 + 2t + odd of the 32-row block
      int64_t ro[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int v = v0 + 2 * t + (odd ? 1 : 0);
        const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        ro[t] = row < d.m ? d.offM[row] : -1;
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (co[j] < 0) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float a0 = val(i, j, v0 + 2 * t), a1 = val(i, j, v0 + 2 * t + 1);
          const int sent = __builtin_bit_cast(int, odd ? a0 : a1);
          // quad_perm [1,0,3,2]: exchange with the neighbouring lane
          const float got = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, sent, 0xB1, 0xF, 0xF, false));
          if (ro[t] >= 0) Cz[ro[t] + co[j]] = odd ? make_float2(got, a1) : make_float2(a0, got);
        }
      }
    }
}

// Store of a wave's 64 x 32 complex block from the 3M products (one 32x32
// accumulator block per 32 rows: T1 = Ar Br, T2 = Ai Bi, T3 = (Ar+Ai)(Br+Bi);
// Re = T1 - T2, Im = T3 - T1 - T2), row-major or through the offset tables.
__device__ __forceinline__ void store_3m(const GemmDesc& d, bool perm, const TileCoord& tc, int wm, int wn, int lane,
                                         const f16v (&t1)[2], const f16v (&t2)[2], const f16v (&t3)[2]) {
  const int h = lane >> 5, l32 = lane & 31;
  if (!perm) {  // row-major [M|N]: addresses from the indices alone
    const int64_t col = tc.col0 + wn * 32 + l32;
    if (col >= d.n) return;
    float2* C = d.C + tc.b * d.m * d.n + col;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < d.m) {
          float2 o;
          o.x = t1[i][v] - t2[i][v];
          o.y = t3[i][v] - t1[i][v] - t2[i][v];
          C[row * d.n] = o;
        }
      }
    return;
  }
  const int64_t co = col_offset(d, perm, tc.col0 + wn * 32 + l32);
  if (co < 0) return;
  float2* C = d.C + tc.b * d.m * d.n + co;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v0 = 0; v0 < 16; v0 += 8) {
      int64_t ro[8];
      row_offsets8(d, perm, tc.row0 + wm * 64 + i * 32, h, v0, ro);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int v = v0 + u;
        if (ro[u] >= 0) {
          float2 o;
          o.x = t1[i][v] - t2[i][v];
          o.y = t3[i][v] - t1[i][v] - t2[i][v];
          C[ro[u]] = o;
        }
      }
    }
}

// ------------------------------------------------------------------ 4M, FP32 MFMA
template <int WM, int WN, int VW>
struct Ops4M {
  using S = Shape<WM, WN>;
  static constexpr bool kSwizzle = false;
  static constexpr int kPW = 1;
  static constexpr size_t kLds = S::lds_f32;
  f16v acc[2][2];

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
  }

  template <class St>
  __device__ __forceinline__ void stage(const St& st, char* lds, int buf, int tid) const {
    float* As = reinterpret_cast<float*>(lds) + buf * (S::BM + S::BNC) * PITCH;
    st.store_f32(As, As + S::BM * PITCH, tid);
  }

  __device__ __forceinline__ void compute(const char* lds, int buf, int wm, int wn, int lane) {
    const float* as = reinterpret_cast<const float*>(lds) + buf * (S::BM + S::BNC) * PITCH;
    const float* bs = as + S::BM * PITCH;
    const int h = lane >> 5, l32 = lane & 31, p = lane & 1;
#pragma unroll
    for (int g = 0; g < BKC / 4; ++g) {
      const int koff = (4 * g + 2 * h) * 2;
      f4 a[2], bt[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const f4*>(as + (wm * 64 + i * 32 + l32) * PITCH + koff);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const f4 r = *reinterpret_cast<const f4*>(bs + (wn * 32 + j * 16 + (l32 >> 1)) * PITCH + koff);
        f4 t;
        t.x = p ? r.y : r.x;
        t.y = p ? r.x : -r.y;
        t.z = p ? r.w : r.z;
        t.w = p ? r.z : -r.w;
        bt[j] = t;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, bt[j].x, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, bt[j].y, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].z, bt[j].z, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].w, bt[j].w, acc[i][j], 0, 0, 0);
        }
    }
  }

  __device__ __forceinline__ void store(const GemmDesc& d, bool perm, const TileCoord& tc, int wm, int wn,
                                        int lane) const {
    const int h = lane >> 5, l32 = lane & 31;
    // real column tc.col0*2 + wn*64 + j*32 + l32: complex column >> 1, re/im by parity
    float* C = reinterpret_cast<float*>(d.C + tc.b * d.m * d.n) + (l32 & 1);
    if (!perm) {  // row-major [M|N]: addresses from the indices alone
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int64_t col = (tc.col0 * 2 + wn * 64 + j * 32 + l32) >> 1;
          if (col >= d.n) continue;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            if (row < d.m) C[2 * (row * d.n + col)] = acc[i][j][v];
          }
        }
      return;
    }
    store_perm_pairs(d, tc, wm, wn, lane, [&](int i, int j, int v) { return acc[i][j][v]; });
  }
};

// ------------------------------------------------------------------ 3M, FP32 MFMA
// LDS rows are unpadded (32 floats) with their eight 16-byte slots permuted
// by row (slot = chunk ^ ((row >> 1) & 7)): the fragment reads of 16 lanes
// (16 consecutive rows, one chunk) and the staging stores of 16 lanes (two
// rows) each hit 16 distinct 4-bank groups, as the padded rows of the other
// kernels do, in 49152 instead of 55296 bytes for the (2,2) tile, so three
// of its workgroups fit a CU (two with padded rows).
template <int WM, int WN, int VW>
struct Ops3M {
  using S = Shape<WM, WN>;
  static constexpr bool kSwizzle = false;
  static constexpr int kPW = 1;
  static constexpr int P3 = 32;  // floats per LDS row
  static constexpr size_t kLds = 2 * (S::BM + S::BNC) * P3 * sizeof(float);
  f16v t1[2], t2[2], t3[2];

  // float offset of float fo (even) of LDS row `row`
  __device__ __forceinline__ static int at(int row, int fo) {
    return row * P3 + ((((fo >> 2) ^ ((row >> 1) & 7)) << 2) | (fo & 3));
  }

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) t1[i][v] = t2[i][v] = t3[i][v] = 0.f;
  }

  template <class St>
  __device__ __forceinline__ static void put(float* base, int row, int idx, const f4& v) {
    float* p = base + at(row, 2 * (idx % St::PER_ROW) * VW);
    if constexpr (VW == 2) {
      *reinterpret_cast<f4*>(p) = v;
    } else {
      p[0] = v.x;
      p[1] = v.y;
    }
  }

  template <class St>
  __device__ __forceinline__ void stage(const St& st, char* lds, int buf, int tid) const {
    float* As = reinterpret_cast<float*>(lds) + buf * (S::BM + S::BNC) * P3;
    float* Bs = As + S::BM * P3;
#pragma unroll
    for (int i = 0; i < St::A_LOADS; ++i) put<St>(As, St::row_a(tid + S::NT * i), tid + S::NT * i, st.a[i]);
#pragma unroll
    for (int i = 0; i < St::B_LOADS; ++i) put<St>(Bs, St::row_b(tid + S::NT * i), tid + S::NT * i, st.b[i]);
  }

  __device__ __forceinline__ void compute(const char* lds, int buf, int wm, int wn, int lane) {
    const float* as = reinterpret_cast<const float*>(lds) + buf * (S::BM + S::BNC) * P3;
    const float* bs = as + S::BM * P3;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int g = 0; g < BKC / 4; ++g) {
      const int koff = (4 * g + 2 * h) * 2;
      const f4 rb = *reinterpret_cast<const f4*>(bs + at(wn * 32 + l32, koff));
      const float bs0 = rb.x + rb.y, bs1 = rb.z + rb.w;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const f4 ra = *reinterpret_cast<const f4*>(as + at(wm * 64 + i * 32 + l32, koff));
        const float as0 = ra.x + ra.y, as1 = ra.z + ra.w;
        t1[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.x, rb.x, t1[i], 0, 0, 0);
        t2[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.y, rb.y, t2[i], 0, 0, 0);
        t3[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(as0, bs0, t3[i], 0, 0, 0);
        t1[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.z, rb.z, t1[i], 0, 0, 0);
        t2[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.w, rb.w, t2[i], 0, 0, 0);
        t3[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(as1, bs1, t3[i], 0, 0, 0);
      }
    }
  }

  __device__ __forceinline__ void store(const GemmDesc& d, bool perm, const TileCoord& tc, int wm, int wn,
                                        int lane) const {
    store_3m(d, perm, tc, wm, wn, lane, t1, t2, t3);
  }
};

// ------------------------------------------------------------------ split BF16x3, 4M form
template <int WM, int WN, int VW>
struct OpsBF16x3 {
  using S = Shape<WM, WN>;
  static constexpr bool kSwizzle = true;
  static constexpr int kPW = 1;
  static constexpr size_t kLds = S::lds_bf16;
  // hi*hi products and the two cross products accumulate separately: the
  // cross terms are ~2^-8 smaller, so their rounding barely adds to that of
  // the main sum
  f16v acc[2][2], accx[2][2];

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = accx[i][j][v] = 0.f;
  }

  __device__ __forceinline__ static const uint16_t* planes(const char* lds, int buf) {
    return reinterpret_cast<const uint16_t*>(lds) + buf * S::BF16_STAGE;
  }

  template <class St>
  __device__ __forceinline__ void stage(const St& st, char* lds, int buf, int tid) const {
    uint16_t* Ah = const_cast<uint16_t*>(planes(lds, buf));
    uint16_t* Al = Ah + S::BM * SPITCH;
    uint16_t* Bh = Al + S::BM * SPITCH;
    uint16_t* Bl = Bh + 2 * S::BNC * SPITCH;
    st.store_split(Ah, Al, Bh, Bl, tid);
  }

  // bf16 MFMA 32x32x16: lane (h, r) supplies 8 consecutive K values of row
  // r (A) or real column r (B'); the stage's 32 real k are two sub-steps,
  // lane half h taking k = 8 * (2s + h) .. +7.
  __device__ __forceinline__ void compute(const char* lds, int buf, int wm, int wn, int lane) {
    const uint16_t* Ah = planes(lds, buf);
    const uint16_t* Al = Ah + S::BM * SPITCH;
    const uint16_t* Bh = Al + S::BM * SPITCH;
    const uint16_t* Bl = Bh + 2 * S::BNC * SPITCH;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int koff = 8 * (2 * s + h);
      s8v ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm * 64 + i * 32 + l32;
        ah[i] = *reinterpret_cast<const s8v*>(Ah + row * SPITCH + koff);
        al[i] = *reinterpret_cast<const s8v*>(Al + row * SPITCH + koff);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = 2 * (wn * 32 + j * 16) + l32;  // real column of B'
        bh[j] = *reinterpret_cast<const s8v*>(Bh + row * SPITCH + koff);
        bl[j] = *reinterpret_cast<const s8v*>(Bl + row * SPITCH + koff);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accx[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, ah[i]),
                                                               __builtin_bit_cast(bf8, bl[j]), accx[i][j], 0, 0, 0);
          accx[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, al[i]),
                                                               __builtin_bit_cast(bf8, bh[j]), accx[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, ah[i]),
                                                              __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
        }
    }
  }

  __device__ __forceinline__ void store(const GemmDesc& d, bool perm, const TileCoord& tc, int wm, int wn,
                                        int lane) const {
    const int h = lane >> 5, l32 = lane & 31;
    float* C = reinterpret_cast<float*>(d.C + tc.b * d.m * d.n) + (l32 & 1);
    if (!perm) {  // row-major [M|N]: addresses from the indices alone
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int64_t col = (tc.col0 * 2 + wn * 64 + j * 32 + l32) >> 1;
          if (col >= d.n) continue;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            if (row < d.m) C[2 * (row * d.n + col)] = acc[i][j][v] + accx[i][j][v];
          }
        }
      return;
    }
    store_perm_pairs(d, tc, wm, wn, lane, [&](int i, int j, int v) { return acc[i][j][v] + accx[i][j][v]; });
  }
};

// ------------------------------------------------------------------ split BF16x3, wide waves
// The same products with each wave covering 64 complex columns (four
// 32-column blocks of the real 4M operand) instead of 32: every A fragment
// read from LDS feeds four blocks instead of two and the workgroup's staging
// (and its split) is shared by twice the MFMA work, so the kernel issues
// about 40 % fewer instructions per MFMA.  The accumulator budget of the
// wider tile allows one accumulator set: hi*hi and the two cross products
// accumulate together (FP32, as in the 4M kernel).
template <int WM, int WN, int VW>
struct OpsBF16x3W {
  using S = Shape<WM, WN, 2>;
  static constexpr bool kSwizzle = true;
  static constexpr int kPW = 2;
  static constexpr size_t kLds = S::lds_bf16;
  f16v acc[2][4];

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
  }

  __device__ __forceinline__ static const uint16_t* planes(const char* lds, int buf) {
    return reinterpret_cast<const uint16_t*>(lds) + buf * S::BF16_STAGE;
  }

  template <class St>
  __device__ __forceinline__ void stage(const St& st, char* lds, int buf, int tid) const {
    uint16_t* Ah = const_cast<uint16_t*>(planes(lds, buf));
    uint16_t* Al = Ah + S::BM * SPITCH;
    uint16_t* Bh = Al + S::BM * SPITCH;
    uint16_t* Bl = Bh + 2 * S::BNC * SPITCH;
    st.store_split(Ah, Al, Bh, Bl, tid);
  }

  // lane (h, r) supplies 8 consecutive K values of row r (A) or real column
  // r (B') per 32x32x16 MFMA, as in OpsBF16x3; this wave's real columns of
  // B' are 128 * wn + 32 * j + r, j = 0..3.
  __device__ __forceinline__ void compute(const char* lds, int buf, int wm, int wn, int lane) {
    const uint16_t* Ah = planes(lds, buf);
    const uint16_t* Al = Ah + S::BM * SPITCH;
    const uint16_t* Bh = Al + S::BM * SPITCH;
    const uint16_t* Bl = Bh + 2 * S::BNC * SPITCH;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int koff = 8 * (2 * s + h);
      s8v ah[2], al[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm * 64 + i * 32 + l32;
        ah[i] = *reinterpret_cast<const s8v*>(Ah + row * SPITCH + koff);
        al[i] = *reinterpret_cast<const s8v*>(Al + row * SPITCH + koff);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 128 * wn + 32 * j + l32;
        const s8v bh = *reinterpret_cast<const s8v*>(Bh + row * SPITCH + koff);
        const s8v bl = *reinterpret_cast<const s8v*>(Bl + row * SPITCH + koff);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, ah[i]),
                                                              __builtin_bit_cast(bf8, bl), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, al[i]),
                                                              __builtin_bit_cast(bf8, bh), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, ah[i]),
                                                              __builtin_bit_cast(bf8, bh), acc[i][j], 0, 0, 0);
        }
      }
    }
  }

  __device__ __forceinline__ void store(const GemmDesc& d, bool perm, const TileCoord& tc, int wm, int wn,
                                        int lane) const {
    const int h = lane >> 5, l32 = lane & 31;
    float* C = reinterpret_cast<float*>(d.C + tc.b * d.m * d.n) + (l32 & 1);
    if (!perm) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t col = (tc.col0 * 2 + wn * 128 + j * 32 + l32) >> 1;
          if (col >= d.n) continue;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            if (row < d.m) C[2 * (row * d.n + col)] = acc[i][j][v];
          }
        }
      return;
    }
    store_perm_pairs<2>(d, tc, wm, wn, lane, [&](int i, int j, int v) { return acc[i][j][v]; });
  }
};

// ------------------------------------------------------------------ split BF16x3, 3M form
// The 3M form's three real products T1 = Ar Br, T2 = Ai Bi, T3 = (Ar+Ai)
// (Br+Bi), each as a_hi b_lo + a_lo b_hi + a_hi b_hi on bf16 MFMA
// 32x32x16 into one FP32 accumulator per product: 9 bf16 products per
// complex product instead of the 4M form's 12.  The sum planes are formed
// in float32 at staging, then split like the others.  A stage (16 complex
// k) holds six unpadded bf16 planes per operand (r, i, s, each hi and lo),
// a row of 16 k in 32 bytes; the row's two 16-byte halves swap places
// every 8 rows (slot = half ^ ((row >> 3) & 1)), so the fragment reads of
// 16 lanes (16 rows, one half) and the 4-byte staging stores of a wave (8
// rows x 8 pairs) hit distinct banks.  The wave tile and the store are the
// complex64 3M form's.
template <int WM, int WN, int VW>
struct Ops3MBF16 {
  using S = Shape<WM, WN>;
  static constexpr bool kSwizzle = false;
  static constexpr int kPW = 1;
  static constexpr int ROWB = 32;  // bytes per plane row
  static constexpr int PLANE_A = S::BM * ROWB, PLANE_B = S::BNC * ROWB;
  static constexpr int STAGE = 6 * (PLANE_A + PLANE_B);
  static constexpr size_t kLds = 2 * STAGE;
  f16v t1[2], t2[2], t3[2];

  // byte offset of k (0..15) in plane row `row`
  __device__ __forceinline__ static int at(int row, int k) {
    return row * ROWB + ((((k >> 3) ^ ((row >> 3) & 1)) << 4) | ((k & 7) << 1));
  }

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) t1[i][v] = t2[i][v] = t3[i][v] = 0.f;
  }

  // planes p = 0..5 (r hi, r lo, i hi, i lo, s hi, s lo) at base + p * plane
  template <class St>
  __device__ __forceinline__ static void put(char* base, int plane, int row, int idx, const f4& v) {
    const int off = at(row, (idx % St::PER_ROW) * VW);
    if constexpr (VW == 2) {  // complex k, k + 1: (re k, im k, re k+1, im k+1)
      uint32_t rh, rl, ih, il, sh, sl;
      bf16_split2(v.x, v.z, rh, rl);
      bf16_split2(v.y, v.w, ih, il);
      bf16_split2(v.x + v.y, v.z + v.w, sh, sl);
      *reinterpret_cast<uint32_t*>(base + off) = rh;
      *reinterpret_cast<uint32_t*>(base + plane + off) = rl;
      *reinterpret_cast<uint32_t*>(base + 2 * plane + off) = ih;
      *reinterpret_cast<uint32_t*>(base + 3 * plane + off) = il;
      *reinterpret_cast<uint32_t*>(base + 4 * plane + off) = sh;
      *reinterpret_cast<uint32_t*>(base + 5 * plane + off) = sl;
    } else {  // one complex value: (re, im) split as a pair, the sum alone
      uint32_t h, l, sh, sl;
      bf16_split2(v.x, v.y, h, l);
      bf16_split2(v.x + v.y, 0.f, sh, sl);
      *reinterpret_cast<uint16_t*>(base + off) = static_cast<uint16_t>(h);
      *reinterpret_cast<uint16_t*>(base + plane + off) = static_cast<uint16_t>(l);
      *reinterpret_cast<uint16_t*>(base + 2 * plane + off) = static_cast<uint16_t>(h >> 16);
      *reinterpret_cast<uint16_t*>(base + 3 * plane + off) = static_cast<uint16_t>(l >> 16);
      *reinterpret_cast<uint16_t*>(base + 4 * plane + off) = static_cast<uint16_t>(sh);
      *reinterpret_cast<uint16_t*>(base + 5 * plane + off) = static_cast<uint16_t>(sl);
    }
  }

  template <class St>
  __device__ __forceinline__ void stage(const St& st, char* lds, int buf, int tid) const {
    char* As = lds + buf * STAGE;
    char* Bs = As + 6 * PLANE_A;
#pragma unroll
    for (int i = 0; i < St::A_LOADS; ++i) put<St>(As, PLANE_A, St::row_a(tid + S::NT * i), tid + S::NT * i, st.a[i]);
#pragma unroll
    for (int i = 0; i < St::B_LOADS; ++i) put<St>(Bs, PLANE_B, St::row_b(tid + S::NT * i), tid + S::NT * i, st.b[i]);
  }

  __device__ __forceinline__ static void mm(f16v& t, const s8v& ah, const s8v& al, const s8v& bh, const s8v& bl) {
    t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, ah), __builtin_bit_cast(bf8, bl), t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, al), __builtin_bit_cast(bf8, bh), t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, ah), __builtin_bit_cast(bf8, bh), t, 0, 0, 0);
  }

  // product p (planes 2p, 2p + 1) of the stage into t
  __device__ __forceinline__ static void product(f16v (&t)[2], const char* ah, const char* bh, int oa0, int oa1,
                                                 int ob) {
    const s8v a0h = *reinterpret_cast<const s8v*>(ah + oa0);
    const s8v a0l = *reinterpret_cast<const s8v*>(ah + PLANE_A + oa0);
    const s8v a1h = *reinterpret_cast<const s8v*>(ah + oa1);
    const s8v a1l = *reinterpret_cast<const s8v*>(ah + PLANE_A + oa1);
    const s8v b_h = *reinterpret_cast<const s8v*>(bh + ob);
    const s8v b_l = *reinterpret_cast<const s8v*>(bh + PLANE_B + ob);
    mm(t[0], a0h, a0l, b_h, b_l);
    mm(t[1], a1h, a1l, b_h, b_l);
  }

  // lane (h, r) supplies k = 8h .. 8h + 7 of row r (A) or column r (B);
  // one product at a time keeps a third of the fragments live
  __device__ __forceinline__ void compute(const char* lds, int buf, int wm, int wn, int lane) {
    const char* As = lds + buf * STAGE;
    const char* Bs = As + 6 * PLANE_A;
    const int h = lane >> 5, l32 = lane & 31;
    const int oa0 = at(wm * 64 + l32, 8 * h), oa1 = at(wm * 64 + 32 + l32, 8 * h);
    const int ob = at(wn * 32 + l32, 8 * h);
    product(t1, As, Bs, oa0, oa1, ob);
    product(t2, As + 2 * PLANE_A, Bs + 2 * PLANE_B, oa0, oa1, ob);
    product(t3, As + 4 * PLANE_A, Bs + 4 * PLANE_B, oa0, oa1, ob);
  }

  __device__ __forceinline__ void store(const GemmDesc& d, bool perm, const TileCoord& tc, int wm, int wn,
                                        int lane) const {
    store_3m(d, perm, tc, wm, wn, lane, t1, t2, t3);
  }
};

// ------------------------------------------------------------------ driver
template <int WM, int WN, int VW, bool CHECK, class Ops>
__device__ __forceinline__ void main_loop(const GemmDesc& d, const float2* A, const float2* B, const TileCoord& tc,
                                          char* lds, Ops& ops, int tid, int wm, int wn, int lane) {
  const int64_t nk = (d.k + BKC - 1) / BKC;
  const int64_t ld = row_stride(d);
  Stage<WM, WN, VW, Ops::kSwizzle, Ops::kPW> st;
  st.template load<CHECK>(A, B, d.m, d.n, d.k, ld, tc.row0, tc.col0, 0, tid);
  ops.stage(st, lds, 0, tid);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) st.template load<CHECK>(A, B, d.m, d.n, d.k, ld, tc.row0, tc.col0, (kt + 1) * BKC, tid);
    ops.compute(lds, buf, wm, wn, lane);
    if (kt + 1 < nk) ops.stage(st, lds, buf ^ 1, tid);
    __syncthreads();
  }
}

// Workgroups per CU the compiler must allow for: two for shapes of up to
// four waves, three for 3M's (2,2) with 16-byte loads (its LDS admits
// three; 168 VGPRs each; the 8-byte-load path needs more registers).
template <template <int, int, int> class OpsT, int WM, int WN, int VW>
constexpr int min_blocks() {
  if constexpr (std::is_same_v<OpsT<2, 2, 2>, Ops3M<2, 2, 2>>)
    if (WM * WN == 4 && VW == 2) return 3;
  return WM * WN <= 4 ? 2 : 1;
}

template <template <int, int, int> class OpsT, int WM, int WN, int VW, bool PERM>
__global__ __launch_bounds__(64 * WM * WN, (min_blocks<OpsT, WM, WN, VW>())) void cgemm_mfma(GemmDesc d, int64_t tiles_m, int64_t tiles_n,
                                                           int64_t total) {
  using S = Shape<WM, WN, OpsT<WM, WN, VW>::kPW>;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const TileCoord tc = map_tile_shared<S::BM, S::BNC>(tiles_m, tiles_n, total);
  int64_t oa, ob;
  batch_offsets(d, tc.b, oa, ob);
  const float2* __restrict__ A = d.A + oa;
  const float2* __restrict__ B = d.B + ob;
  OpsT<WM, WN, VW> ops;
  ops.init();
  const bool interior = tc.row0 + S::BM <= d.m && tc.col0 + S::BNC <= d.n && d.k % BKC == 0;
  if (interior)
    main_loop<WM, WN, VW, false>(d, A, B, tc, lds, ops, tid, wm, wn, lane);
  else
    main_loop<WM, WN, VW, true>(d, A, B, tc, lds, ops, tid, wm, wn, lane);
  ops.store(d, PERM, tc, wm, wn, lane);
}

// Persistent grouped form: workgroups loop over the tiles of every entry of
// the table.  Tiles are dealt to the 8 XCDs in contiguous ranges (tiles of
// one entry stay on few XCDs, whose L2 they share) and each workgroup of an
// XCD takes every nb-th tile of its range.  The tile's work is the
// single-GEMM kernel's, line for line.  The tile loop keeps more values
// live than one tile does, so most instances are built for one workgroup
// per CU, which lets the compiler keep accumulators in AGPRs instead of
// spilling (the persistent grid runs a fixed number of workgroups anyway);
// the complex64 (2,2) tile fits two.
template <template <int, int, int> class OpsT, int WM, int WN>
constexpr int grouped_min_blocks() {
  return WM * WN == 4 && !std::is_same_v<OpsT<2, 2, 2>, OpsBF16x3<2, 2, 2>> ? 2 : 1;
}

template <template <int, int, int> class OpsT, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN, (grouped_min_blocks<OpsT, WM, WN>())) void cgemm_mfma_grouped(
    const GroupedEntry* __restrict__ tab, int n, int64_t total) {
  using S = Shape<WM, WN, OpsT<WM, WN, 2>::kPW>;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t per = (total + 7) >> 3;  // tiles per XCD
  const int64_t xcd = blockIdx.x & 7, nb = gridDim.x >> 3;
  for (int64_t q = blockIdx.x >> 3; q < per; q += nb) {
    const int64_t t = xcd * per + q;
    if (t >= total) break;
    int e = 0;
    while (e + 1 < n && tab[e + 1].tile0 <= t) ++e;
    const GemmDesc& d = tab[e].d;
    const TileCoord tc = tile_of<S::BM, S::BNC>(t - tab[e].tile0, tab[e].tiles_m, tab[e].tiles_n);
    int64_t oa, ob;
    batch_offsets(d, tc.b, oa, ob);
    const float2* __restrict__ A = d.A + oa;
    const float2* __restrict__ B = d.B + ob;
    OpsT<WM, WN, 2> ops;
    ops.init();
    const bool interior = tc.row0 + S::BM <= d.m && tc.col0 + S::BNC <= d.n && d.k % BKC == 0;
    if (interior)
      main_loop<WM, WN, 2, false>(d, A, B, tc, lds, ops, tid, wm, wn, lane);
    else
      main_loop<WM, WN, 2, true>(d, A, B, tc, lds, ops, tid, wm, wn, lane);
    ops.store(d, d.offM != nullptr, tc, wm, wn, lane);
  }
}

// ------------------------------------------ split-bf16x3 on pre-split planes
// Large split-precision steps split each operand once, into bf16 planes in
// global memory, instead of in the staging of every workgroup that reads
// it.  A row of A (or of the 4M real operand B': row 2c = (br, -bi, ...),
// row 2c + 1 = (bi, br, ...)) is stored in blocks of 16 complex k, 128
// bytes = [32 bf16 hi | 32 bf16 lo] of its 32 floats; rows are padded to
// the tile and k to 16 with zeros, so staging needs no bounds tests and
// moves blocks straight from global memory into LDS (16 bytes per lane,
// global_load_lds_dwordx4: no registers and no VALU on the way).  The split
// is the staging kernels' (round to nearest even, lo = rne(x - hi)) and the
// tile's products and accumulation order are those of OpsBF16x3W, so the
// result is bitwise that of the wide-wave kernel.
//
// LDS: two stages of four unpadded planes (256 rows x 64 bytes each); the
// four 16-byte slots of a row are permuted by row (slot = chunk ^ ((row >> 2)
// & 3)), so that the fragment reads of 16 lanes (16 rows, one chunk) hit 16
// distinct 4-bank groups.  Each stage has one barrier, in its middle: the
// waves issue the first half's MFMAs (whose fragments they read during the
// previous half) and read the second half's fragments, then meet; after the
// barrier the stage's loads two stages ahead go out into the buffer just
// released, the next stage's first fragments are read, and the second
// half's MFMAs run, their issue interleaved with those reads.
constexpr int PS_PLANE = 256 * 64;        // bytes of one LDS plane
constexpr int PS_STAGE = 4 * PS_PLANE;    // A hi, A lo, B' hi, B' lo
constexpr size_t PS_LDS = 2 * PS_STAGE;   // 128 KiB

// uint32 (bf16 pair) index of the hi half of complex element (row, kc) in
// planes of kp complex columns; the lo half is 16 further
__device__ __forceinline__ int64_t ps_index(int64_t row, int64_t kc, int64_t kp) {
  return row * 2 * kp + 32 * (kc >> 4) + (kc & 15);
}

__device__ __forceinline__ void ps_split(float x, float y, uint32_t& hi, uint32_t& lo) {
  Stage<4, 2, 2, true, 2>::split2(x, y, hi, lo);
}

// One thread per complex element of the padded planes; 16 consecutive
// threads cover one 128-byte block (their loads 128 contiguous bytes of
// the row, their stores the block).
__global__ __launch_bounds__(256) void split_planes_a(const float2* __restrict__ X, int64_t rows, int64_t k,
                                                     int64_t ld, uint32_t nkb, uint32_t blocks, int64_t kp,
                                                     uint32_t* __restrict__ out) {
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < blocks * 16u; t += gridDim.x * 256u) {
    const uint32_t b = t >> 4, e = t & 15;
    const int64_t row = b / nkb, kc = int64_t{b % nkb} * 16 + e;
    uint64_t v = 0;
    if (row < rows && kc < k) v = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(X + row * ld + kc));
    uint32_t hi, lo;
    ps_split(__uint_as_float(static_cast<uint32_t>(v)), __uint_as_float(static_cast<uint32_t>(v >> 32)), hi, lo);
    const int64_t p = ps_index(row, kc, kp);
    __builtin_nontemporal_store(hi, out + p);
    __builtin_nontemporal_store(lo, out + p + 16);
  }
}

// B -> the planes of B' (two real rows per complex row of B; negating a
// bf16 flips its sign bit, swapping re/im rotates the packed pair).
__global__ __launch_bounds__(256) void split_planes_b(const float2* __restrict__ X, int64_t rows, int64_t k,
                                                     int64_t ld, uint32_t nkb, uint32_t blocks, int64_t kp,
                                                     uint32_t* __restrict__ out) {
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < blocks * 16u; t += gridDim.x * 256u) {
    const uint32_t b = t >> 4, e = t & 15;
    const int64_t row = b / nkb, kc = int64_t{b % nkb} * 16 + e;
    uint64_t v = 0;
    if (row < rows && kc < k) v = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(X + row * ld + kc));
    uint32_t hi, lo;
    ps_split(__uint_as_float(static_cast<uint32_t>(v)), __uint_as_float(static_cast<uint32_t>(v >> 32)), hi, lo);
    const int64_t p0 = ps_index(2 * row, kc, kp), p1 = p0 + 2 * kp;
    __builtin_nontemporal_store(hi ^ 0x80000000u, out + p0);
    __builtin_nontemporal_store(lo ^ 0x80000000u, out + p0 + 16);
    __builtin_nontemporal_store((hi >> 16) | (hi << 16), out + p1);
    __builtin_nontemporal_store((lo >> 16) | (lo << 16), out + p1 + 16);
  }
}

// 3M form: the real parts X_r, X_i and X_s = X_r + X_i (float32 sums) of
// a complex operand as three real matrices of `rows` x k, each in the
// planes layout of a real GEMM (blocks of 32 real k, [32 bf16 hi | 32 bf16
// lo], kp real k pairs per row; padding rows and k zero).  One thread per
// pair of real k (two complex elements) of a padded row; P points at the
// r planes, the i and s planes follow at `plane` uint32 apart.
__global__ __launch_bounds__(256) void split_planes_3m(const float2* __restrict__ X, int64_t rows, int64_t k,
                                                      int64_t ld, uint32_t kp, uint32_t pairs, int64_t plane,
                                                      uint32_t* __restrict__ P) {
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < pairs; t += gridDim.x * 256u) {
    const int64_t row = t / kp, q = t - row * kp;  // real k 2q, 2q + 1
    float2 x0 = make_float2(0.f, 0.f), x1 = x0;
    if (row < rows) {
      const float2* src = X + row * ld + 2 * q;
      if (2 * q < k) x0 = src[0];
      if (2 * q + 1 < k) x1 = src[1];
    }
    uint32_t rh, rl, ih, il, sh, sl;
    ps_split(x0.x, x1.x, rh, rl);
    ps_split(x0.y, x1.y, ih, il);
    ps_split(x0.x + x0.y, x1.x + x1.y, sh, sl);
    const int64_t o = ps_index(row, q, kp);
    __builtin_nontemporal_store(rh, P + o);
    __builtin_nontemporal_store(rl, P + o + 16);
    __builtin_nontemporal_store(ih, P + plane + o);
    __builtin_nontemporal_store(il, P + plane + o + 16);
    __builtin_nontemporal_store(sh, P + 2 * plane + o);
    __builtin_nontemporal_store(sl, P + 2 * plane + o + 16);
  }
}

// C from the three real products (rows of `ldt` floats, T2 and T3 `tplane`
// floats after T1): re = T1 - T2, im = T3 - T1 - T2 in float32, the same
// expressions as the 3M store; row-major or through the offset tables.
__global__ __launch_bounds__(256) void combine_3m(const float* __restrict__ T, int64_t tplane, int64_t ldt,
                                                 GemmDesc d) {
  const int64_t total = d.m * d.n;
  const double inv_n = 1.0 / static_cast<double>(d.n);
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * 256) {
    const int64_t row = plane_row(e, d.n, inv_n), col = e - row * d.n;
    const int64_t o = row * ldt + col;
    const float t1 = T[o], t2 = T[tplane + o], t3 = T[2 * tplane + o];
    float2 v;
    v.x = t1 - t2;
    v.y = t3 - t1 - t2;
    const int64_t c = d.offM ? d.offM[row] + d.offN[col] : e;
    d.C[c] = v;
  }
}

struct PsFrag {
  s8v ah[2], al[2], bh[4], bl[4];
};

// Fragments of sub-step s (16 real k) for wave (wm, wn), as OpsBF16x3W
// reads them: lane (h, r) takes 8 consecutive k of row r (A) or real column
// r (B').
__device__ __forceinline__ void ps_read(const char* stage, int wm, int wn, int h, int l32, int s, PsFrag& f) {
  const int ch = 2 * s + h;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = wm * 64 + i * 32 + l32;
    const int off = row * 64 + 16 * (ch ^ ((row >> 2) & 3));
    f.ah[i] = *reinterpret_cast<const s8v*>(stage + off);
    f.al[i] = *reinterpret_cast<const s8v*>(stage + PS_PLANE + off);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = 128 * wn + 32 * j + l32;
    const int off = row * 64 + 16 * (ch ^ ((row >> 2) & 3));
    f.bh[j] = *reinterpret_cast<const s8v*>(stage + 2 * PS_PLANE + off);
    f.bl[j] = *reinterpret_cast<const s8v*>(stage + 3 * PS_PLANE + off);
  }
}

// OpsBF16x3W's products in its order: per block, a_hi b_lo, a_lo b_hi, a_hi b_hi
__device__ __forceinline__ void ps_mfma(f16v (&acc)[2][4], const PsFrag& f) {
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, f.ah[i]),
                                                          __builtin_bit_cast(bf8, f.bl[j]), acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, f.al[i]),
                                                          __builtin_bit_cast(bf8, f.bh[j]), acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, f.ah[i]),
                                                          __builtin_bit_cast(bf8, f.bh[j]), acc[i][j], 0, 0, 0);
    }
}

// Stage kk's blocks of the tile into LDS buffer `buf`: 64 wave-loads of 1
// KiB (16 rows x 4 slots of one plane), 8 per wave.  `wave` is uniform.
__device__ __forceinline__ void ps_issue(char* lds, int buf, int64_t kk, const uint32_t* gA, const uint32_t* gB,
                                         int64_t kp, int wave, int lane) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int bid = wave * 8 + q;
    const int plane = bid >> 4, rb = bid & 15;
    const int row = rb * 16 + (lane >> 2), slot = lane & 3;
    const int c = slot ^ ((row >> 2) & 3);
    const uint32_t* g = (plane < 2 ? gA : gB) + row * 2 * kp + 2 * kk + 16 * (plane & 1) + 4 * c;
    char* dst = lds + buf * PS_STAGE + plane * PS_PLANE + rb * 1024;
    __builtin_amdgcn_global_load_lds(static_cast<const void*>(g), (__attribute__((address_space(3))) void*)dst, 16, 0,
                                     0);
  }
}

// One K stage (16 complex k).  ISSUE: load stage kt + 2 after the barrier;
// READ: read the next stage's first fragments into f0.
template <bool ISSUE, bool READ>
__device__ __forceinline__ void ps_stage(f16v (&acc)[2][4], PsFrag& f0, PsFrag& f1, char* lds, int64_t kt,
                                         const uint32_t* gA, const uint32_t* gB, int64_t kp, int wave, int lane,
                                         int wm, int wn, int h, int l32) {
  const int buf = kt & 1;
  ps_read(lds + buf * PS_STAGE, wm, wn, h, l32, 1, f1);
  ps_mfma(acc, f0);
#pragma unroll
  for (int r = 0; r < 12; ++r) {  // one fragment read per two MFMAs
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
  }
  __builtin_amdgcn_s_waitcnt(0);  // this wave's reads done, stage kt + 1 landed
  __syncthreads();
  if constexpr (ISSUE) ps_issue(lds, buf, (kt + 2) * BKC, gA, gB, kp, wave, lane);
  if constexpr (READ) ps_read(lds + (buf ^ 1) * PS_STAGE, wm, wn, h, l32, 0, f0);
  ps_mfma(acc, f1);
  if constexpr (ISSUE) __builtin_amdgcn_sched_group_barrier(0x020, 8, 0);
  if constexpr (READ) {
#pragma unroll
    for (int r = 0; r < 12; ++r) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
    }
  }
}

// gfx9 s_waitcnt immediate: vmcnt <= 8, expcnt and lgkmcnt not waited for
constexpr int kWaitVm8 = 0x0F78;

template <bool PERM>
__global__ __launch_bounds__(512, 1) void cgemm_bf16x3_presplit(GemmDesc d, const uint32_t* __restrict__ Ap,
                                                                const uint32_t* __restrict__ Bp, int64_t kp,
                                                                int64_t tiles_m, int64_t tiles_n, int64_t total) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  const TileCoord tc = map_tile_shared<kPresplitBM, kPresplitBNC>(tiles_m, tiles_n, total);
  const uint32_t* gA = Ap + tc.row0 * 2 * kp;
  const uint32_t* gB = Bp + 2 * tc.col0 * 2 * kp;
  const int64_t nk = kp / BKC;
  OpsBF16x3W<4, 2, 2> ops;
  ops.init();
  PsFrag f0, f1;
  ps_issue(lds, 0, 0, gA, gB, kp, wave, lane);
  if (nk > 1) {
    ps_issue(lds, 1, BKC, gA, gB, kp, wave, lane);
    __builtin_amdgcn_s_waitcnt(kWaitVm8);  // stage 0 landed (loads complete in order)
  } else {
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  ps_read(lds, wm, wn, h, l32, 0, f0);
  if (nk > 1) {
    for (int64_t kt = 0; kt + 2 < nk; ++kt)
      ps_stage<true, true>(ops.acc, f0, f1, lds, kt, gA, gB, kp, wave, lane, wm, wn, h, l32);
    ps_stage<false, true>(ops.acc, f0, f1, lds, nk - 2, gA, gB, kp, wave, lane, wm, wn, h, l32);
  }
  ps_stage<false, false>(ops.acc, f0, f1, lds, nk - 1, gA, gB, kp, wave, lane, wm, wn, h, l32);
  ops.store(d, PERM, tc, wm, wn, lane);
}

// LDS above 64 KiB for the pre-split kernel, once per device.
hipError_t ensure_lds_presplit() {
  static std::atomic<uint64_t> attr_set{0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = uint64_t{1} << (dev & 63);
  if (attr_set.load(std::memory_order_acquire) & bit) return hipSuccess;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(cgemm_bf16x3_presplit<false>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(PS_LDS));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(cgemm_bf16x3_presplit<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(PS_LDS));
  if (e == hipSuccess) attr_set.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

// LDS above 64 KiB must be allowed per kernel, once per device (done for
// every instance when a context is created, so that no first launch inside
// a graph capture has to do it).
template <template <int, int, int> class OpsT, int WM, int WN, int VW, bool PERM>
hipError_t ensure_lds(size_t lds) {
  static std::atomic<uint64_t> attr_set{0};
  if (lds <= 65536) return hipSuccess;
  int dev = 0;
  const hipError_t ge = hipGetDevice(&dev);
  if (ge != hipSuccess) return ge;
  const uint64_t bit = uint64_t{1} << (dev & 63);
  if (attr_set.load(std::memory_order_acquire) & bit) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(cgemm_mfma<OpsT, WM, WN, VW, PERM>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e == hipSuccess) attr_set.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

template <template <int, int, int> class OpsT, int WM, int WN, int VW, bool PERM>
hipError_t launch_one(const GemmDesc& d, size_t lds, hipStream_t s) {
  using S = Shape<WM, WN, OpsT<WM, WN, VW>::kPW>;
  const int64_t tiles_m = (d.m + S::BM - 1) / S::BM;
  const int64_t tiles_n = (d.n + S::BNC - 1) / S::BNC;
  const int64_t total = tiles_m * tiles_n * d.h;
  // one workgroup per tile; the grid's work-items must fit 32 bits
  if (total * S::NT > 0xFFFFFFFFLL) return hipErrorInvalidValue;
  const hipError_t e = ensure_lds<OpsT, WM, WN, VW, PERM>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((cgemm_mfma<OpsT, WM, WN, VW, PERM>), dim3(static_cast<unsigned>(total)), dim3(S::NT), lds, s, d,
                     tiles_m, tiles_n, total);
  return hipGetLastError();
}

template <template <int, int, int> class OpsT, int WM, int WN>
hipError_t ensure_lds_grouped(size_t lds) {
  static std::atomic<uint64_t> attr_set{0};
  if (lds <= 65536) return hipSuccess;
  int dev = 0;
  const hipError_t ge = hipGetDevice(&dev);
  if (ge != hipSuccess) return ge;
  const uint64_t bit = uint64_t{1} << (dev & 63);
  if (attr_set.load(std::memory_order_acquire) & bit) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(cgemm_mfma_grouped<OpsT, WM, WN>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e == hipSuccess) attr_set.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

template <template <int, int, int> class OpsT, int WM, int WN, bool GROUPED = true>
void prepare_shape(bool) {
  const size_t lds = OpsT<WM, WN, 2>::kLds;
  (void)ensure_lds<OpsT, WM, WN, 2, false>(lds);
  (void)ensure_lds<OpsT, WM, WN, 2, true>(lds);
  if constexpr (GROUPED) (void)ensure_lds_grouped<OpsT, WM, WN>(lds);
}

// Persistent grid: a multiple of 8 (one range of tiles per XCD), never more
// than the tiles; at most 512 workgroups (two per compute unit), or 2048
// waves for the shapes of fewer than four waves.
template <template <int, int, int> class OpsT, int WM, int WN>
hipError_t launch_grouped_shape(const GroupedEntry* tab, int n, int64_t total, bool, hipStream_t s) {
  using S = Shape<WM, WN, OpsT<WM, WN, 2>::kPW>;
  const size_t lds = OpsT<WM, WN, 2>::kLds;
  const hipError_t e = ensure_lds_grouped<OpsT, WM, WN>(lds);
  if (e != hipSuccess) return e;
  constexpr int64_t cap = WM * WN < 4 ? 2048 / (WM * WN) : 512;
  int64_t grid = (total + 7) / 8 * 8;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL((cgemm_mfma_grouped<OpsT, WM, WN>), dim3(static_cast<unsigned>(grid)), dim3(S::NT), lds, s, tab,
                     n, total);
  return hipGetLastError();
}

// Grouped forms are built only where the persistent tile loop fits the
// registers without spilling (compiler resource report for gfx950, with
// the launch bounds above): every complex64 4M shape, 3M but (4,4), and
// split precision's (2,2), (1,2), (2,1), (1,1).  Other grouped launches fail
// with hipErrorInvalidValue; callers run those GEMMs one launch each.
template <template <int, int, int> class OpsT>
constexpr bool grouped_ok(int variant) {
  if (variant < 0 || variant >= kGemmVariants) return false;
  if constexpr (std::is_same_v<OpsT<2, 2, 2>, OpsBF16x3<2, 2, 2>>) return variant == 0 || variant >= 4;
  if constexpr (std::is_same_v<OpsT<2, 2, 2>, Ops3M<2, 2, 2>>) return variant != 3;
  if constexpr (std::is_same_v<OpsT<2, 2, 2>, Ops3MBF16<2, 2, 2>>) return variant != 3;
  return true;
}

template <template <int, int, int> class OpsT>
hipError_t launch_grouped_variant(const GroupedEntry* tab, int n, int64_t total, int variant, bool bf16,
                                  hipStream_t s) {
  if (!grouped_ok<OpsT>(variant)) return hipErrorInvalidValue;
  switch (variant) {
    case 0: return launch_grouped_shape<OpsT, 2, 2>(tab, n, total, bf16, s);
    case 4: return launch_grouped_shape<OpsT, 1, 2>(tab, n, total, bf16, s);
    case 5: return launch_grouped_shape<OpsT, 2, 1>(tab, n, total, bf16, s);
    case 6: return launch_grouped_shape<OpsT, 1, 1>(tab, n, total, bf16, s);
    default: break;
  }
  if constexpr (!std::is_same_v<OpsT<2, 2, 2>, OpsBF16x3<2, 2, 2>>) {
    switch (variant) {
      case 1: return launch_grouped_shape<OpsT, 4, 2>(tab, n, total, bf16, s);
      case 2: return launch_grouped_shape<OpsT, 2, 4>(tab, n, total, bf16, s);
      case 3:
        if constexpr (!std::is_same_v<OpsT<2, 2, 2>, Ops3M<2, 2, 2>> && !std::is_same_v<OpsT<2, 2, 2>, Ops3MBF16<2, 2, 2>>)
          return launch_grouped_shape<OpsT, 4, 4>(tab, n, total, bf16, s);
        break;
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// The narrow split tile has no (4,4) instance: split precision runs that
// tile size as 4x2 wide waves (the narrow waves' two accumulator sets would
// spill).  Nor has the 3M split form: its three accumulator sets spill at
// sixteen waves per workgroup (compiler resource report), so a forced
// variant 3 runs its (4,2) tile.
template <template <int, int, int> class OpsT>
constexpr bool is_split() {
  return std::is_same_v<OpsT<2, 2, 2>, OpsBF16x3<2, 2, 2>>;
}
template <template <int, int, int> class OpsT>
constexpr bool is_split_3m() {
  return std::is_same_v<OpsT<2, 2, 2>, Ops3MBF16<2, 2, 2>>;
}

template <template <int, int, int> class OpsT>
void prepare_ops(bool bf16) {
  prepare_shape<OpsT, 2, 2, grouped_ok<OpsT>(0)>(bf16);
  prepare_shape<OpsT, 4, 2, grouped_ok<OpsT>(1)>(bf16);
  prepare_shape<OpsT, 2, 4, grouped_ok<OpsT>(2)>(bf16);
  if constexpr (!is_split<OpsT>() && !is_split_3m<OpsT>()) prepare_shape<OpsT, 4, 4, grouped_ok<OpsT>(3)>(bf16);
  prepare_shape<OpsT, 1, 2, grouped_ok<OpsT>(4)>(bf16);
  prepare_shape<OpsT, 2, 1, grouped_ok<OpsT>(5)>(bf16);
  prepare_shape<OpsT, 1, 1, grouped_ok<OpsT>(6)>(bf16);
  const size_t lds = OpsT<2, 2, 1>::kLds;  // odd-k path
  (void)ensure_lds<OpsT, 2, 2, 1, false>(lds);
  (void)ensure_lds<OpsT, 2, 2, 1, true>(lds);
}

template <template <int, int, int> class OpsT, int WM, int WN>
hipError_t launch_shape(const GemmDesc& d, bool, hipStream_t s) {
  const size_t lds = OpsT<WM, WN, 2>::kLds;
  const bool perm = d.offM != nullptr;
  return perm ? launch_one<OpsT, WM, WN, 2, true>(d, lds, s) : launch_one<OpsT, WM, WN, 2, false>(d, lds, s);
}

template <template <int, int, int> class OpsT>
hipError_t launch_variant(const GemmDesc& d, int variant, bool bf16, hipStream_t s) {
  if ((d.k | row_stride(d)) % 2 != 0) {  // odd k or row stride: 8-byte loads, default shape only
    const size_t lds = OpsT<2, 2, 1>::kLds;
    return d.offM ? launch_one<OpsT, 2, 2, 1, true>(d, lds, s) : launch_one<OpsT, 2, 2, 1, false>(d, lds, s);
  }
  // split precision: the 256 x 128 tile runs as 4x2 wide waves (16 waves of
  // the narrow kind would spill their two accumulator sets)
  switch (variant) {
    case 0: return launch_shape<OpsT, 2, 2>(d, bf16, s);
    case 1: return launch_shape<OpsT, 4, 2>(d, bf16, s);
    case 2: return launch_shape<OpsT, 2, 4>(d, bf16, s);
    case 3:
      if constexpr (is_split<OpsT>()) return launch_shape<OpsBF16x3W, 4, 2>(d, true, s);
      else if constexpr (is_split_3m<OpsT>()) return launch_shape<OpsT, 4, 2>(d, true, s);
      else return launch_shape<OpsT, 4, 4>(d, bf16, s);
    case 4: return launch_shape<OpsT, 1, 2>(d, bf16, s);
    case 5: return launch_shape<OpsT, 2, 1>(d, bf16, s);
    case 6: return launch_shape<OpsT, 1, 1>(d, bf16, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

void prepare_gemm_kernels() {
  prepare_ops<Ops4M>(false);
  prepare_ops<Ops3M>(false);
  prepare_ops<OpsBF16x3>(true);
  prepare_ops<Ops3MBF16>(true);
  prepare_shape<OpsBF16x3W, 4, 2, false>(true);
  (void)ensure_lds_presplit();
}

void gemm_variant_tile(int variant, int* bm, int* bnc) {
  static const int wm[kGemmVariants] = {2, 4, 2, 4, 1, 2, 1};
  static const int wn[kGemmVariants] = {2, 2, 4, 4, 2, 1, 1};
  if (variant < 0 || variant >= kGemmVariants) variant = 0;
  *bm = 64 * wm[variant];
  *bnc = 32 * wn[variant];
}

int64_t grouped_layout(GroupedEntry* e, int n, int variant) {
  int bm = 0, bnc = 0;
  gemm_variant_tile(variant, &bm, &bnc);
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    const GemmDesc& d = e[i].d;
    if (d.h <= 0 || d.m <= 0 || d.n <= 0 || d.k <= 0 || (d.k | row_stride(d)) % 2 != 0) return 0;
    e[i].tiles_m = (d.m + bm - 1) / bm;
    e[i].tiles_n = (d.n + bnc - 1) / bnc;
    e[i].tile0 = total;
    total += e[i].tiles_m * e[i].tiles_n * d.h;
  }
  return total;
}

bool grouped_variant_ok(Form form, Prec prec, int variant) {
  if (prec == Prec::BF16X3)
    return form == Form::M3 ? grouped_ok<Ops3MBF16>(variant) : grouped_ok<OpsBF16x3>(variant);
  return form == Form::M3 ? grouped_ok<Ops3M>(variant) : grouped_ok<Ops4M>(variant);
}

hipError_t launch_gemm_grouped(const GroupedEntry* dev, int n, int64_t total, int variant, Form form, Prec prec,
                               hipStream_t s) {
  if (n <= 0 || total <= 0) return hipSuccess;
  if (prec == Prec::BF16X3)
    return form == Form::M3 ? launch_grouped_variant<Ops3MBF16>(dev, n, total, variant, true, s)
                            : launch_grouped_variant<OpsBF16x3>(dev, n, total, variant, true, s);
  if (form == Form::M3) return launch_grouped_variant<Ops3M>(dev, n, total, variant, false, s);
  return launch_grouped_variant<Ops4M>(dev, n, total, variant, false, s);
}

hipError_t launch_gemm_presplit(const GemmDesc& d, void* planes, bool have_a, bool have_b, hipStream_t s) {
  if (d.h <= 0 || d.m <= 0 || d.n <= 0) return hipSuccess;
  if (d.k <= 0 || d.h != 1 || d.rowA || d.kA || d.rowB || d.kB || !planes ||
      reinterpret_cast<uintptr_t>(planes) % 256 != 0)
    return hipErrorInvalidValue;
  const int64_t mp = presplit_rows_a(d.m), np2 = presplit_rows_b(d.n), kp = presplit_k(d.k);
  const int64_t nkb = kp / 16;
  // one thread per padded element, counted in 32 bits
  if ((mp > np2 / 2 ? mp : np2 / 2) * kp >= (int64_t{1} << 31)) return hipErrorInvalidValue;
  const hipError_t e = ensure_lds_presplit();
  if (e != hipSuccess) return e;
  uint32_t* Ap = static_cast<uint32_t*>(planes);
  uint32_t* Bp = Ap + mp * 2 * kp;
  const int64_t ld = row_stride(d);
  auto grid = [](int64_t threads) {
    const int64_t g = (threads + 255) / 256;
    return static_cast<unsigned>(g < 131072 ? g : 131072);
  };
  const uint32_t blocks_a = static_cast<uint32_t>(mp * nkb), blocks_b = static_cast<uint32_t>(np2 / 2 * nkb);
  if (!have_a)
    hipLaunchKernelGGL(split_planes_a, dim3(grid(int64_t{blocks_a} * 16)), dim3(256), 0, s, d.A, d.m, d.k, ld,
                       static_cast<uint32_t>(nkb), blocks_a, kp, Ap);
  if (!have_b)
    hipLaunchKernelGGL(split_planes_b, dim3(grid(int64_t{blocks_b} * 16)), dim3(256), 0, s, d.B, d.n, d.k, ld,
                       static_cast<uint32_t>(nkb), blocks_b, kp, Bp);
  const int64_t tiles_m = mp / kPresplitBM, tiles_n = np2 / 2 / kPresplitBNC, total = tiles_m * tiles_n;
  if (d.offM)
    hipLaunchKernelGGL(cgemm_bf16x3_presplit<true>, dim3(static_cast<unsigned>(total)), dim3(512), PS_LDS, s, d, Ap,
                       Bp, kp, tiles_m, tiles_n, total);
  else
    hipLaunchKernelGGL(cgemm_bf16x3_presplit<false>, dim3(static_cast<unsigned>(total)), dim3(512), PS_LDS, s, d, Ap,
                       Bp, kp, tiles_m, tiles_n, total);
  return hipGetLastError();
}

hipError_t launch_gemm_presplit_3m(const GemmDesc& d, void* buf, bool have_a, bool have_b, hipStream_t s) {
  if (d.h <= 0 || d.m <= 0 || d.n <= 0) return hipSuccess;
  if (d.k <= 0 || d.h != 1 || d.rowA || d.kA || d.rowB || d.kB || !buf || reinterpret_cast<uintptr_t>(buf) % 256 != 0)
    return hipErrorInvalidValue;
  const Presplit3M g = presplit_3m_layout(d.m, d.n, d.k);
  // one thread per real k pair of a padded row, counted in 32 bits
  if ((g.mp > g.np ? g.mp : g.np) * g.kp >= (int64_t{1} << 31)) return hipErrorInvalidValue;
  hipError_t e = ensure_lds_presplit();
  if (e != hipSuccess) return e;
  char* base = static_cast<char*>(buf);
  uint32_t* Ap = reinterpret_cast<uint32_t*>(base);
  uint32_t* Bp = reinterpret_cast<uint32_t*>(base + g.off_b);
  float* T = reinterpret_cast<float*>(base + g.off_t);
  const int64_t ld = row_stride(d);
  auto grid = [](int64_t threads) {
    const int64_t q = (threads + 255) / 256;
    return static_cast<unsigned>(q < 131072 ? q : 131072);
  };
  const int64_t plane_a = g.mp * 2 * g.kp, plane_b = g.np * 2 * g.kp;  // uint32 per plane
  if (!have_a)
    hipLaunchKernelGGL(split_planes_3m, dim3(grid(g.mp * g.kp)), dim3(256), 0, s, d.A, d.m, d.k, ld,
                       static_cast<uint32_t>(g.kp), static_cast<uint32_t>(g.mp * g.kp), plane_a, Ap);
  if (!have_b)
    hipLaunchKernelGGL(split_planes_3m, dim3(grid(g.np * g.kp)), dim3(256), 0, s, d.B, d.n, d.k, ld,
                       static_cast<uint32_t>(g.kp), static_cast<uint32_t>(g.np * g.kp), plane_b, Bp);
  // T_p = X_p Y_p^T as the pre-split kernel's real GEMM: m rows, np real
  // columns (nh column pairs), 2 kp real k; stored row-major in pairs
  const int64_t tiles_m = g.mp / kPresplitBM, tiles_n = g.np / 2 / kPresplitBNC, total = tiles_m * tiles_n;
  for (int p = 0; p < 3; ++p) {
    GemmDesc dp;
    std::memset(&dp, 0, sizeof(dp));
    dp.C = reinterpret_cast<float2*>(T + p * g.tplane);
    dp.m = d.m;
    dp.n = g.nh;
    dp.k = g.kp;
    dp.h = 1;
    hipLaunchKernelGGL(cgemm_bf16x3_presplit<false>, dim3(static_cast<unsigned>(total)), dim3(512), PS_LDS, s, dp,
                       Ap + p * plane_a, Bp + p * plane_b, g.kp, tiles_m, tiles_n, total);
  }
  hipLaunchKernelGGL(combine_3m, dim3(grid(d.m * d.n)), dim3(256), 0, s, T, g.tplane, 2 * g.nh, d);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmDesc& d, GemmKernel kind, int variant, Form form, Prec prec, hipStream_t s) {
  if (d.h <= 0 || d.m <= 0 || d.n <= 0) return hipSuccess;
  if (d.k <= 0) return hipErrorInvalidValue;
  if (kind != GemmKernel::MFMA) return launch_gemm_valu(d, kind, prec, s);
  if (prec == Prec::BF16X3)
    return form == Form::M3 ? launch_variant<Ops3MBF16>(d, variant, true, s)
                            : launch_variant<OpsBF16x3>(d, variant, true, s);
  if (form == Form::M3) return launch_variant<Ops3M>(d, variant, false, s);
  return launch_variant<Ops4M>(d, variant, false, s);
}

}  // namespace tnc
