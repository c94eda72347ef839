// Batched complex GEMM kernels for gfx950:  C[b,i,j] = sum_l A[b,i,l] B[b,j,l].
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
// a_hi b_hi + a_hi b_lo + a_lo b_hi on bf16 MFMA with FP32 accumulation.
//
// Tiling: a 256-thread workgroup (4 wave64) owns a 128 x 64 complex tile of
// C; each wave owns 64 x 32 complex.  K advances 16 complex per stage
// through double-buffered LDS (rows padded to 144 B so the 16-byte fragment
// reads of 16 lanes hit 16 distinct 4-bank groups).  Workgroups are remapped
// so that consecutive tiles land on one XCD (the hardware deals workgroups
// round-robin over the 8 XCDs, each with its own L2) and tiles sweep the
// N dimension in groups of 8 M-tiles for L2 reuse.
#include "kernels.hpp"

namespace tnc {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));

constexpr int BM = 128;    // rows of C per workgroup
constexpr int BNC = 64;    // complex columns of C per workgroup
constexpr int BKC = 16;    // complex k per LDS stage
constexpr int PITCH = 36;  // floats per LDS row (32 data + 4 pad)
constexpr int GROUP_M = 8;

__device__ __forceinline__ void batch_offsets(const GemmDesc& d, int64_t b, int64_t& oa, int64_t& ob) {
  oa = 0;
  ob = 0;
  if (d.pow2) {
    for (int j = d.nbd - 1; j >= 0; --j) {
      const int64_t dig = b & (static_cast<int64_t>(d.bext[j]) - 1);
      b >>= d.bshift[j];
      oa += dig * d.bsA[j];
      ob += dig * d.bsB[j];
    }
  } else {
    for (int j = d.nbd - 1; j >= 0; --j) {
      const int64_t e = d.bext[j];
      const int64_t q = b / e;
      const int64_t dig = b - q * e;
      b = q;
      oa += dig * d.bsA[j];
      ob += dig * d.bsB[j];
    }
  }
}

struct TileCoord {
  int64_t b, row0, col0;
};

__device__ __forceinline__ TileCoord map_tile(int64_t tiles_m, int64_t tiles_n, int64_t total) {
  int64_t wg = blockIdx.x;
  const int64_t per = total >> 3;
  if (wg < (per << 3)) wg = (wg & 7) * per + (wg >> 3);
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

// Global -> register staging of one K stage (VW complex per load).
template <int VW>
struct Stage {
  static constexpr int A_LOADS = BM * BKC / VW / 256;
  static constexpr int B_LOADS = BNC * BKC / VW / 256;
  static constexpr int PER_ROW = BKC / VW;
  f4 a[A_LOADS > 0 ? A_LOADS : 1];
  f4 b[B_LOADS > 0 ? B_LOADS : 1];

  __device__ __forceinline__ void load(const float2* __restrict__ A, const float2* __restrict__ B,
                                       int64_t m, int64_t n, int64_t k, int64_t row0, int64_t col0,
                                       int64_t kk, int tid) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int idx = tid + 256 * i;
      const int r = idx / PER_ROW;
      const int c = (idx % PER_ROW) * VW;
      const int64_t gr = row0 + r, gk = kk + c;
      f4 v = {0.f, 0.f, 0.f, 0.f};
      if (gr < m && gk < k) {
        const float2* p = A + gr * k + gk;
        if constexpr (VW == 2) {
          v = *reinterpret_cast<const f4*>(p);
        } else {
          const float2 x = *p;
          v.x = x.x;
          v.y = x.y;
        }
      }
      a[i] = v;
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int idx = tid + 256 * i;
      const int r = idx / PER_ROW;
      const int c = (idx % PER_ROW) * VW;
      const int64_t gr = col0 + r, gk = kk + c;
      f4 v = {0.f, 0.f, 0.f, 0.f};
      if (gr < n && gk < k) {
        const float2* p = B + gr * k + gk;
        if constexpr (VW == 2) {
          v = *reinterpret_cast<const f4*>(p);
        } else {
          const float2 x = *p;
          v.x = x.x;
          v.y = x.y;
        }
      }
      b[i] = v;
    }
  }

  __device__ __forceinline__ void store(float* As, float* Bs, int tid) const {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int idx = tid + 256 * i;
      const int r = idx / PER_ROW;
      const int c = (idx % PER_ROW) * VW;
      float* p = As + r * PITCH + 2 * c;
      if constexpr (VW == 2) {
        *reinterpret_cast<f4*>(p) = a[i];
      } else {
        p[0] = a[i].x;
        p[1] = a[i].y;
      }
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int idx = tid + 256 * i;
      const int r = idx / PER_ROW;
      const int c = (idx % PER_ROW) * VW;
      float* p = Bs + r * PITCH + 2 * c;
      if constexpr (VW == 2) {
        *reinterpret_cast<f4*>(p) = b[i];
      } else {
        p[0] = b[i].x;
        p[1] = b[i].y;
      }
    }
  }
};

__device__ __forceinline__ int64_t c_index(const GemmDesc& d, bool perm, int64_t b, int64_t row, int64_t col) {
  return b * d.m * d.n + (perm ? d.offM[row] + d.offN[col] : row * d.n + col);
}

// ------------------------------------------------------------------ 4M, FP32 MFMA
template <int VW, bool PERM>
__global__ __launch_bounds__(256) void cgemm_4m_mfma(GemmDesc d, int64_t tiles_m, int64_t tiles_n,
                                                      int64_t total) {
  __shared__ __attribute__((aligned(16))) float As[2][BM * PITCH];
  __shared__ __attribute__((aligned(16))) float Bs[2][BNC * PITCH];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31, p = lane & 1;
  const TileCoord tc = map_tile(tiles_m, tiles_n, total);
  int64_t oa, ob;
  batch_offsets(d, tc.b, oa, ob);
  const float2* __restrict__ A = d.A + oa;
  const float2* __restrict__ B = d.B + ob;

  f16v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  const int64_t nk = (d.k + BKC - 1) / BKC;
  Stage<VW> st;
  st.load(A, B, d.m, d.n, d.k, tc.row0, tc.col0, 0, tid);
  st.store(As[0], Bs[0], tid);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) st.load(A, B, d.m, d.n, d.k, tc.row0, tc.col0, (kt + 1) * BKC, tid);
    const float* as = As[buf];
    const float* bs = Bs[buf];
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
    if (kt + 1 < nk) st.store(As[buf ^ 1], Bs[buf ^ 1], tid);
    __syncthreads();
  }

  float* C = reinterpret_cast<float*>(d.C);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t ncr = tc.col0 * 2 + wn * 64 + j * 32 + l32;  // real column
      const int64_t col = ncr >> 1;
      if (col >= d.n) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < d.m) C[2 * c_index(d, PERM, tc.b, row, col) + (ncr & 1)] = acc[i][j][v];
      }
    }
}

// ------------------------------------------------------------------ 3M, FP32 MFMA
template <int VW, bool PERM>
__global__ __launch_bounds__(256) void cgemm_3m_mfma(GemmDesc d, int64_t tiles_m, int64_t tiles_n,
                                                      int64_t total) {
  __shared__ __attribute__((aligned(16))) float As[2][BM * PITCH];
  __shared__ __attribute__((aligned(16))) float Bs[2][BNC * PITCH];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  const TileCoord tc = map_tile(tiles_m, tiles_n, total);
  int64_t oa, ob;
  batch_offsets(d, tc.b, oa, ob);
  const float2* __restrict__ A = d.A + oa;
  const float2* __restrict__ B = d.B + ob;

  f16v t1[2], t2[2], t3[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) t1[i][v] = t2[i][v] = t3[i][v] = 0.f;

  const int64_t nk = (d.k + BKC - 1) / BKC;
  Stage<VW> st;
  st.load(A, B, d.m, d.n, d.k, tc.row0, tc.col0, 0, tid);
  st.store(As[0], Bs[0], tid);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) st.load(A, B, d.m, d.n, d.k, tc.row0, tc.col0, (kt + 1) * BKC, tid);
    const float* as = As[buf];
    const float* bs = Bs[buf];
#pragma unroll
    for (int g = 0; g < BKC / 4; ++g) {
      const int koff = (4 * g + 2 * h) * 2;
      const f4 rb = *reinterpret_cast<const f4*>(bs + (wn * 32 + l32) * PITCH + koff);
      const float br0 = rb.x, bi0 = rb.y, br1 = rb.z, bi1 = rb.w;
      const float bs0 = br0 + bi0, bs1 = br1 + bi1;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const f4 ra = *reinterpret_cast<const f4*>(as + (wm * 64 + i * 32 + l32) * PITCH + koff);
        const float as0 = ra.x + ra.y, as1 = ra.z + ra.w;
        t1[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.x, br0, t1[i], 0, 0, 0);
        t2[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.y, bi0, t2[i], 0, 0, 0);
        t3[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(as0, bs0, t3[i], 0, 0, 0);
        t1[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.z, br1, t1[i], 0, 0, 0);
        t2[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra.w, bi1, t2[i], 0, 0, 0);
        t3[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(as1, bs1, t3[i], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) st.store(As[buf ^ 1], Bs[buf ^ 1], tid);
    __syncthreads();
  }

  const int64_t col = tc.col0 + wn * 32 + l32;
  if (col < d.n) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < d.m) {
          float2 o;
          o.x = t1[i][v] - t2[i][v];
          o.y = t3[i][v] - t1[i][v] - t2[i][v];
          d.C[c_index(d, PERM, tc.b, row, col)] = o;
        }
      }
  }
}

// ------------------------------------------------------------------ split BF16x3, 4M form
__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u & 0xFFFF0000u;
}

// hi/lo bf16 halves (as 16-bit patterns) of one float32.
__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
  const uint32_t h = bf16_rne_bits(x);
  const float r = x - __uint_as_float(h);
  hi = static_cast<uint16_t>(h >> 16);
  lo = static_cast<uint16_t>(bf16_rne_bits(r) >> 16);
}

// LDS layout for the split kernel: for each of A and B, a hi plane and a lo
// plane, each row = 2*BKC bf16 of the real-expanded K (32 values = 64 B)
// padded to 80 B.  Rows of B hold B's interleaved values unexpanded; the
// re/im select and sign flip are applied to the bf16 fragments.
constexpr int SPITCH = 40;  // uint16 per LDS row (32 data + 8 pad)

template <int VW, bool PERM>
__global__ __launch_bounds__(256) void cgemm_4m_bf16x3(GemmDesc d, int64_t tiles_m, int64_t tiles_n,
                                                        int64_t total) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[2][BM * SPITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Al[2][BM * SPITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[2][BNC * SPITCH];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[2][BNC * SPITCH];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31, p = lane & 1;
  const TileCoord tc = map_tile(tiles_m, tiles_n, total);
  int64_t oa, ob;
  batch_offsets(d, tc.b, oa, ob);
  const float2* __restrict__ A = d.A + oa;
  const float2* __restrict__ B = d.B + ob;

  // hi*hi products and the two cross products accumulate separately: the
  // cross terms are ~2^-8 smaller, so their rounding barely adds to that of
  // the main sum
  f16v acc[2][2], accx[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = accx[i][j][v] = 0.f;

  auto store_split = [&](const Stage<VW>& st, int buf) {
#pragma unroll
    for (int i = 0; i < Stage<VW>::A_LOADS; ++i) {
      const int idx = tid + 256 * i;
      const int r = idx / Stage<VW>::PER_ROW;
      const int c = (idx % Stage<VW>::PER_ROW) * VW;
      uint16_t hi[4], lo[4];
      split_bf16(st.a[i].x, hi[0], lo[0]);
      split_bf16(st.a[i].y, hi[1], lo[1]);
      split_bf16(st.a[i].z, hi[2], lo[2]);
      split_bf16(st.a[i].w, hi[3], lo[3]);
      for (int e = 0; e < 2 * VW; ++e) {
        Ah[buf][r * SPITCH + 2 * c + e] = hi[e];
        Al[buf][r * SPITCH + 2 * c + e] = lo[e];
      }
    }
#pragma unroll
    for (int i = 0; i < Stage<VW>::B_LOADS; ++i) {
      const int idx = tid + 256 * i;
      const int r = idx / Stage<VW>::PER_ROW;
      const int c = (idx % Stage<VW>::PER_ROW) * VW;
      uint16_t hi[4], lo[4];
      split_bf16(st.b[i].x, hi[0], lo[0]);
      split_bf16(st.b[i].y, hi[1], lo[1]);
      split_bf16(st.b[i].z, hi[2], lo[2]);
      split_bf16(st.b[i].w, hi[3], lo[3]);
      for (int e = 0; e < 2 * VW; ++e) {
        Bh[buf][r * SPITCH + 2 * c + e] = hi[e];
        Bl[buf][r * SPITCH + 2 * c + e] = lo[e];
      }
    }
  };

  // The bf16 MFMA 32x32x16: lane (h, r) supplies 8 consecutive K values of
  // row r; here K = the 32 real k' of one stage, lane half h taking
  // k' = 8*(2s + h) .. +7 for sub-step s in {0, 1}.
  const int64_t nk = (d.k + BKC - 1) / BKC;
  Stage<VW> st;
  st.load(A, B, d.m, d.n, d.k, tc.row0, tc.col0, 0, tid);
  store_split(st, 0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) st.load(A, B, d.m, d.n, d.k, tc.row0, tc.col0, (kt + 1) * BKC, tid);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int koff = 8 * (2 * s + h);
      s8v ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm * 64 + i * 32 + l32;
        ah[i] = *reinterpret_cast<const s8v*>(&Ah[buf][row * SPITCH + koff]);
        al[i] = *reinterpret_cast<const s8v*>(&Al[buf][row * SPITCH + koff]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = wn * 32 + j * 16 + (l32 >> 1);
        const s8v rh = *reinterpret_cast<const s8v*>(&Bh[buf][row * SPITCH + koff]);
        const s8v rl = *reinterpret_cast<const s8v*>(&Bl[buf][row * SPITCH + koff]);
        s8v th, tl;
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          // pair (re, im) of one complex k; p = 0 -> (re, -im), p = 1 -> (im, re)
          const short hre = rh[e], him = rh[e + 1], lre = rl[e], lim = rl[e + 1];
          th[e] = p ? him : hre;
          th[e + 1] = p ? hre : static_cast<short>(him ^ static_cast<short>(0x8000));
          tl[e] = p ? lim : lre;
          tl[e + 1] = p ? lre : static_cast<short>(lim ^ static_cast<short>(0x8000));
        }
        bh[j] = th;
        bl[j] = tl;
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
    if (kt + 1 < nk) store_split(st, buf ^ 1);
    __syncthreads();
  }

  float* C = reinterpret_cast<float*>(d.C);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t ncr = tc.col0 * 2 + wn * 64 + j * 32 + l32;
      const int64_t col = ncr >> 1;
      if (col >= d.n) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = tc.row0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < d.m) C[2 * c_index(d, PERM, tc.b, row, col) + (ncr & 1)] = acc[i][j][v] + accx[i][j][v];
      }
    }
}

// ------------------------------------------------------------------ small shapes (VALU)
__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(bf16_rne_bits(x)); }

// a*b with both factors split: hi = a_hi b_hi, cross = a_hi b_lo + a_lo b_hi
// (each product exact in FP32).
__device__ __forceinline__ void split_mul(float a, float b, float& hi, float& cross) {
  const float ah = bf16_round(a), al = bf16_round(a - ah);
  const float bh = bf16_round(b), bl = bf16_round(b - bh);
  hi = ah * bh;
  cross = ah * bl + al * bh;
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void cgemm_small(GemmDesc d) {
  const int64_t mn = d.m * d.n;
  const int64_t total = d.h * mn;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t b = idx / mn;
    const int64_t r = idx - b * mn;
    const int64_t i = r / d.n;
    const int64_t j = r - i * d.n;
    int64_t oa, ob;
    batch_offsets(d, b, oa, ob);
    const float2* a = d.A + oa + i * d.k;
    const float2* bb = d.B + ob + j * d.k;
    float cr = 0.f, ci = 0.f, crx = 0.f, cix = 0.f;
    for (int64_t l = 0; l < d.k; ++l) {
      const float2 x = a[l];
      const float2 y = bb[l];
      if constexpr (SPLIT) {
        float h1, x1, h2, x2, h3, x3, h4, x4;
        split_mul(x.x, y.x, h1, x1);
        split_mul(x.y, y.y, h2, x2);
        split_mul(x.x, y.y, h3, x3);
        split_mul(x.y, y.x, h4, x4);
        cr += h1;
        cr -= h2;
        ci += h3;
        ci += h4;
        crx += x1 - x2;
        cix += x3 + x4;
      } else {
        cr = fmaf(x.x, y.x, cr);
        cr = fmaf(-x.y, y.y, cr);
        ci = fmaf(x.x, y.y, ci);
        ci = fmaf(x.y, y.x, ci);
      }
    }
    const int64_t c = b * mn + (d.offM ? d.offM[i] + d.offN[j] : r);
    d.C[c] = make_float2(cr + crx, ci + cix);
  }
}

// Long reductions with few outputs (k large, m*n tiny): one wave64 per output
// element; lanes stride over k with coalesced reads and the 64 partial sums
// are combined by a fixed butterfly, so the summation error grows like
// (k/64 + 6) roundings instead of k.
template <bool SPLIT>
__global__ __launch_bounds__(256) void cgemm_dot(GemmDesc d) {
  const int lane = threadIdx.x & 63;
  const int64_t mn = d.m * d.n;
  const int64_t total = d.h * mn;
  const int64_t out = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (out >= total) return;  // uniform per wave
  const int64_t b = out / mn;
  const int64_t r = out - b * mn;
  const int64_t i = r / d.n;
  const int64_t j = r - i * d.n;
  int64_t oa, ob;
  batch_offsets(d, b, oa, ob);
  const float2* a = d.A + oa + i * d.k;
  const float2* bb = d.B + ob + j * d.k;
  float cr = 0.f, ci = 0.f, crx = 0.f, cix = 0.f;
  for (int64_t l = lane; l < d.k; l += 64) {
    const float2 x = a[l];
    const float2 y = bb[l];
    if constexpr (SPLIT) {
      float h1, x1, h2, x2, h3, x3, h4, x4;
      split_mul(x.x, y.x, h1, x1);
      split_mul(x.y, y.y, h2, x2);
      split_mul(x.x, y.y, h3, x3);
      split_mul(x.y, y.x, h4, x4);
      cr += h1;
      cr -= h2;
      ci += h3;
      ci += h4;
      crx += x1 - x2;
      cix += x3 + x4;
    } else {
      cr = fmaf(x.x, y.x, cr);
      cr = fmaf(-x.y, y.y, cr);
      ci = fmaf(x.x, y.y, ci);
      ci = fmaf(x.y, y.x, ci);
    }
  }
  cr += crx;
  ci += cix;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    cr += __shfl_xor(cr, off, 64);
    ci += __shfl_xor(ci, off, 64);
  }
  if (lane == 0) {
    const int64_t c = b * mn + (d.offM ? d.offM[i] + d.offN[j] : r);
    d.C[c] = make_float2(cr, ci);
  }
}

}  // namespace

hipError_t launch_gemm(const GemmDesc& d, GemmKernel kind, Form form, Prec prec, hipStream_t s) {
  if (d.h <= 0 || d.m <= 0 || d.n <= 0) return hipSuccess;
  if (d.k <= 0) return hipErrorInvalidValue;
  if (kind == GemmKernel::DOT) {
    const int64_t total = d.h * d.m * d.n;
    const int64_t grid = (total + 3) / 4;
    if (grid > 0x7FFFFFLL) return hipErrorInvalidValue;
    if (prec == Prec::BF16X3)
      hipLaunchKernelGGL(cgemm_dot<true>, dim3(grid), dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL(cgemm_dot<false>, dim3(grid), dim3(256), 0, s, d);
    return hipGetLastError();
  }
  if (kind == GemmKernel::SMALL) {
    const int64_t total = d.h * d.m * d.n;
    int64_t grid = (total + 255) / 256;
    if (grid > 1048576) grid = 1048576;
    if (prec == Prec::BF16X3)
      hipLaunchKernelGGL(cgemm_small<true>, dim3(grid), dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL(cgemm_small<false>, dim3(grid), dim3(256), 0, s, d);
    return hipGetLastError();
  }
  const int64_t tiles_m = (d.m + BM - 1) / BM;
  const int64_t tiles_n = (d.n + BNC - 1) / BNC;
  const int64_t total = tiles_m * tiles_n * d.h;
  // one workgroup per tile; the grid's x extent times 256 must fit 32 bits
  if (total > (1LL << 24) - 1) return hipErrorInvalidValue;
  const bool vec2 = (d.k % 2) == 0;
  const bool perm = d.offM != nullptr;
  const dim3 grid(static_cast<unsigned>(total)), block(256);
#define TNC_GEMM_LAUNCH(KERN)                                                                 \
  do {                                                                                        \
    if (vec2 && perm)                                                                         \
      hipLaunchKernelGGL((KERN<2, true>), grid, block, 0, s, d, tiles_m, tiles_n, total);     \
    else if (vec2)                                                                            \
      hipLaunchKernelGGL((KERN<2, false>), grid, block, 0, s, d, tiles_m, tiles_n, total);    \
    else if (perm)                                                                            \
      hipLaunchKernelGGL((KERN<1, true>), grid, block, 0, s, d, tiles_m, tiles_n, total);     \
    else                                                                                      \
      hipLaunchKernelGGL((KERN<1, false>), grid, block, 0, s, d, tiles_m, tiles_n, total);    \
  } while (0)
  if (prec == Prec::BF16X3)
    TNC_GEMM_LAUNCH(cgemm_4m_bf16x3);
  else if (form == Form::M3)
    TNC_GEMM_LAUNCH(cgemm_3m_mfma);
  else
    TNC_GEMM_LAUNCH(cgemm_4m_mfma);
#undef TNC_GEMM_LAUNCH
  return hipGetLastError();
}

}  // namespace tnc
