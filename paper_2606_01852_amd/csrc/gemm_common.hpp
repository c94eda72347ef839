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

}  // namespace tnc
