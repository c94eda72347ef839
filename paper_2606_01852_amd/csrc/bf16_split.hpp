// Split of float pairs into bf16 hi/lo halves (device, internal): hi =
// round-to-nearest-even of x (the hardware conversion of two floats at a
// time, packed [first | second << 16]), lo = rne(x - hi), where x - hi is
// exact in float32.  Shared by the GEMMs' staging, the pre-split planes and
// the permutes that write planes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tnc {

__device__ __forceinline__ void bf16_split2(float x, float y, uint32_t& hi, uint32_t& lo) {
  typedef float fv2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bv2 __attribute__((ext_vector_type(2)));
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector((fv2){x, y}, bv2));
  const float rx = x - __uint_as_float(hi << 16);
  const float ry = y - __uint_as_float(hi & 0xFFFF0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((fv2){rx, ry}, bv2));
}

// Planes of split operands (rows of blocks of 16 complex k, 128 bytes =
// [32 bf16 hi | 32 bf16 lo]) for an operand stored densely as rows of k
// complex values, k a multiple of 16.  Element o = row * k + kc:
//   A planes:  hi pair at 2 o - (o & 15), lo pair 16 further;
//   B' planes: real rows 2 row (re, -im) and 2 row + 1 (im, re), i.e. the
//              hi pair of row 2 row at 2 (o + row k) - (o & 15), of row
//              2 row + 1 at 2 k further, lo pairs 16 further.
// Row of element o in rows of k (k > 0, o < 2^52): the quotient through a
// double reciprocal is within one of o / k and one correction step each way
// makes it exact (no 64-bit integer division in the kernels).
__device__ __forceinline__ int64_t plane_row(int64_t o, int64_t k, double inv_k) {
  int64_t r = static_cast<int64_t>(static_cast<double>(o) * inv_k);
  const int64_t rem = o - r * k;
  return r + (rem >= k) - (rem < 0);
}

__device__ __forceinline__ uint32_t swap_halves(uint32_t x) { return (x >> 16) | (x << 16); }

__device__ __forceinline__ void put_planes_a(uint32_t* P, int64_t o, float re, float im) {
  uint32_t hi, lo;
  bf16_split2(re, im, hi, lo);
  const int64_t p = 2 * o - (o & 15);
  __builtin_nontemporal_store(hi, P + p);
  __builtin_nontemporal_store(lo, P + p + 16);
}

__device__ __forceinline__ void put_planes_b(uint32_t* P, int64_t o, int64_t k, double inv_k, float re, float im) {
  uint32_t hi, lo;
  bf16_split2(re, im, hi, lo);
  const int64_t row = plane_row(o, k, inv_k);
  const int64_t p0 = 2 * (o + row * k) - (o & 15), p1 = p0 + 2 * k;
  __builtin_nontemporal_store(hi ^ 0x80000000u, P + p0);
  __builtin_nontemporal_store(lo ^ 0x80000000u, P + p0 + 16);
  __builtin_nontemporal_store(swap_halves(hi), P + p1);
  __builtin_nontemporal_store(swap_halves(lo), P + p1 + 16);
}

// Two adjacent elements o, o + 1 (o even, so both sit in one block of 16
// and, k being a multiple of 16, in one row): their hi pairs are adjacent,
// as are their lo pairs, so each plane takes one 8-byte store and eight
// lanes with consecutive pairs fill a whole 128-byte block.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void put_planes_a2(uint32_t* P, int64_t o, float re0, float im0, float re1,
                                              float im1) {
  uint32_t h0, l0, h1, l1;
  bf16_split2(re0, im0, h0, l0);
  bf16_split2(re1, im1, h1, l1);
  const int64_t p = 2 * o - (o & 15);
  __builtin_nontemporal_store(u32x2{h0, h1}, reinterpret_cast<u32x2*>(P + p));
  __builtin_nontemporal_store(u32x2{l0, l1}, reinterpret_cast<u32x2*>(P + p + 16));
}

__device__ __forceinline__ void put_planes_b2(uint32_t* P, int64_t o, int64_t k, double inv_k, float re0, float im0,
                                              float re1, float im1) {
  uint32_t h0, l0, h1, l1;
  bf16_split2(re0, im0, h0, l0);
  bf16_split2(re1, im1, h1, l1);
  const int64_t row = plane_row(o, k, inv_k);
  const int64_t p0 = 2 * (o + row * k) - (o & 15), p1 = p0 + 2 * k;
  const uint32_t s = 0x80000000u;
  __builtin_nontemporal_store(u32x2{h0 ^ s, h1 ^ s}, reinterpret_cast<u32x2*>(P + p0));
  __builtin_nontemporal_store(u32x2{l0 ^ s, l1 ^ s}, reinterpret_cast<u32x2*>(P + p0 + 16));
  __builtin_nontemporal_store(u32x2{swap_halves(h0), swap_halves(h1)}, reinterpret_cast<u32x2*>(P + p1));
  __builtin_nontemporal_store(u32x2{swap_halves(l0), swap_halves(l1)}, reinterpret_cast<u32x2*>(P + p1 + 16));
}

// 3M form: the planes of three real GEMM operands X_r, X_i and X_s =
// X_r + X_i (float32 sums) for an operand stored densely as rows of k
// complex values, k a multiple of 32 (then a row is k / 32 blocks of 32 real
// k, [32 bf16 hi | 32 bf16 lo], k uint32 per row with no padding).  Element
// o = row * k + kc is real k kc of its row: bf16 pair q = kc / 2 of the row,
// half kc & 1 of it; the i and s planes follow the r planes at `plane`
// uint32 apart.
__device__ __forceinline__ int64_t planes_3m_index(int64_t row, int64_t kc, int64_t k) {
  const int64_t q = kc >> 1;
  return row * k + 32 * (q >> 4) + (q & 15);
}

__device__ __forceinline__ void put_planes_3m(uint32_t* P, int64_t o, int64_t k, double inv_k, int64_t plane,
                                              float re, float im) {
  const int64_t row = plane_row(o, k, inv_k), kc = o - row * k;
  const int64_t h = 2 * planes_3m_index(row, kc, k) + (kc & 1);  // bf16 index of the hi half
  uint16_t* Q = reinterpret_cast<uint16_t*>(P);
  uint32_t rh, rl, ih, il;
  bf16_split2(re, im, rh, rl);
  bf16_split2(re + im, 0.f, ih, il);  // the s plane's pair (its low half)
  __builtin_nontemporal_store(static_cast<uint16_t>(rh), Q + h);
  __builtin_nontemporal_store(static_cast<uint16_t>(rl), Q + h + 32);
  __builtin_nontemporal_store(static_cast<uint16_t>(rh >> 16), Q + 2 * plane + h);
  __builtin_nontemporal_store(static_cast<uint16_t>(rl >> 16), Q + 2 * plane + h + 32);
  __builtin_nontemporal_store(static_cast<uint16_t>(ih), Q + 4 * plane + h);
  __builtin_nontemporal_store(static_cast<uint16_t>(il), Q + 4 * plane + h + 32);
}

// Two adjacent elements o, o + 1 (o even): one bf16 pair of each plane.
__device__ __forceinline__ void put_planes_3m2(uint32_t* P, int64_t o, int64_t k, double inv_k, int64_t plane,
                                               float re0, float im0, float re1, float im1) {
  const int64_t row = plane_row(o, k, inv_k);
  const int64_t i = planes_3m_index(row, o - row * k, k);
  uint32_t rh, rl, ih, il, sh, sl;
  bf16_split2(re0, re1, rh, rl);
  bf16_split2(im0, im1, ih, il);
  bf16_split2(re0 + im0, re1 + im1, sh, sl);
  __builtin_nontemporal_store(rh, P + i);
  __builtin_nontemporal_store(rl, P + i + 16);
  __builtin_nontemporal_store(ih, P + plane + i);
  __builtin_nontemporal_store(il, P + plane + i + 16);
  __builtin_nontemporal_store(sh, P + 2 * plane + i);
  __builtin_nontemporal_store(sl, P + 2 * plane + i + 16);
}

}  // namespace tnc
