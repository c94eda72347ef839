// Device helpers shared by the complex-GEMM kernels (internal).
#pragma once

#include "kernels.hpp"

namespace tnc {

// Offsets of batch entry b in A and B: b is row-major over the descriptor's
// batch dims; each digit times that dim's stride (0 broadcasts the operand).
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

// Round-to-nearest-even float32 -> bf16 -> float32 (the hardware
// conversion; bit-identical to clearing the low 16 bits after adding
// 0x7FFF + the lowest kept bit).
__device__ __forceinline__ float bf16_round(float x) { return static_cast<float>(static_cast<__bf16>(x)); }

// a*b with both factors split: hi = a_hi b_hi, cross = a_hi b_lo + a_lo b_hi
// (each product exact in float32).
__device__ __forceinline__ void split_mul(float a, float b, float& hi, float& cross) {
  const float ah = bf16_round(a), al = bf16_round(a - ah);
  const float bh = bf16_round(b), bl = bf16_round(b - bh);
  hi = ah * bh;
  cross = ah * bl + al * bh;
}

// c += x * y for one complex product, in the fixed order the one-thread-
// per-output kernels use (split precision: hi products into cr/ci, cross
// products into crx/cix).
template <bool SPLIT>
__device__ __forceinline__ void cmac(float2 x, float2 y, float& cr, float& ci, float& crx, float& cix) {
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

// sum over l < k of A[l] * B[l], accumulated in order l = 0, 1, ...: the
// elements are loaded four at a time ahead of their products (eight loads
// in flight instead of two per step of a latency-bound loop); the rounding
// sequence is that of the plain loop.
template <bool SPLIT>
__device__ __forceinline__ void cdot_serial(const float2* A, const float2* B, int64_t k, float& cr, float& ci,
                                            float& crx, float& cix) {
  int64_t l = 0;
  for (; l + 4 <= k; l += 4) {
    float2 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = A[l + u];
      y[u] = B[l + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) cmac<SPLIT>(x[u], y[u], cr, ci, crx, cix);
  }
  for (; l < k; ++l) cmac<SPLIT>(A[l], B[l], cr, ci, crx, cix);
}

// The same sum with operands read through tables (an operand without
// tables is K-contiguous at a0 / b0): element l of the A row at
// a0[kA[l]], of the B row at b0[kB[l]]; the accumulation order is that of
// cdot_serial, so the result is bitwise the one of contiguous copies.
template <bool SPLIT>
__device__ __forceinline__ void cdot_tables(const float2* a0, const int64_t* kA, const float2* b0, const int64_t* kB,
                                            int64_t k, float& cr, float& ci, float& crx, float& cix) {
  for (int64_t l = 0; l < k; ++l) {
    const float2 x = kA ? a0[kA[l]] : a0[l];
    const float2 y = kB ? b0[kB[l]] : b0[l];
    cmac<SPLIT>(x, y, cr, ci, crx, cix);
  }
}

}  // namespace tnc
