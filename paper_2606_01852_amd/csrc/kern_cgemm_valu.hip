// Complex GEMM kernels for shapes that do not fill MFMA tiles (VALU): the
// same pairwise-contraction-as-GEMM of Sec. II-B for steps with few
// outputs or tiny extents.
//
// cgemm_small: one thread per output element, k looped in order; used for
// the many tiny steps of circuit networks (m, n or k of a few elements).
// cgemm_dot:   one wave64 per output element for long reductions with few
// outputs (k large, m*n tiny); 4 x 64 partial sums are combined by a fixed
// tree, so the summation error grows like k/256 + 8 roundings, not k.
// Both honour the split-bf16 precision with the same products as the MFMA
// kernel (hi*hi and the two cross products accumulated separately).
#include "gemm_common.hpp"

namespace tnc {

namespace {

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
    float cr = 0.f, ci = 0.f, crx = 0.f, cix = 0.f;
    if (d.kA || d.kB) {
      const float2* a = d.A + oa + (d.baseA ? *d.baseA : 0) + (d.rowA ? d.rowA[i] : i * row_stride(d));
      const float2* bb = d.B + ob + (d.baseB ? *d.baseB : 0) + (d.rowB ? d.rowB[j] : j * row_stride(d));
      cdot_tables<SPLIT>(a, d.kA, bb, d.kB, d.k, cr, ci, crx, cix);
    } else {
      cdot_serial<SPLIT>(d.A + oa + i * row_stride(d), d.B + ob + j * row_stride(d), d.k, cr, ci, crx, cix);
    }
    const int64_t c = b * mn + (d.offM ? d.offM[i] + d.offN[j] : r);
    if constexpr (SPLIT)
      d.C[c] = make_float2(cr + crx, ci + cix);
    else
      d.C[c] = make_float2(cr, ci);
  }
}

// Long reductions with few outputs (k large, m*n tiny): one wave64 per output
// element; lanes stride over k with coalesced reads, each lane keeping four
// independent partial sums (four loads per operand in flight), and the
// 64 x 4 partial sums are combined by a fixed tree, so the summation error
// grows like (k/256 + 8) roundings instead of k.
template <bool SPLIT>
struct DotAcc {
  float cr = 0.f, ci = 0.f, crx = 0.f, cix = 0.f;
  __device__ __forceinline__ void add(float2 x, float2 y) { cmac<SPLIT>(x, y, cr, ci, crx, cix); }
};

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
  const float2* a = d.A + oa + i * row_stride(d);
  const float2* bb = d.B + ob + j * row_stride(d);
  DotAcc<SPLIT> acc[4];
  int64_t l = lane;
  for (; l + 192 < d.k; l += 256) {
    float2 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = a[l + 64 * u];
      y[u] = bb[l + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u].add(x[u], y[u]);
  }
#pragma unroll
  for (int u = 0; u < 3; ++u)  // the last < 256 elements
    if (l + 64 * u < d.k) acc[u].add(a[l + 64 * u], bb[l + 64 * u]);
  float cr[4], ci[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    cr[u] = acc[u].cr + acc[u].crx;
    ci[u] = acc[u].ci + acc[u].cix;
  }
  float sr = (cr[0] + cr[1]) + (cr[2] + cr[3]);
  float si = (ci[0] + ci[1]) + (ci[2] + ci[3]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if (lane == 0) {
    const int64_t c = b * mn + (d.offM ? d.offM[i] + d.offN[j] : r);
    d.C[c] = make_float2(sr, si);
  }
}

__global__ __launch_bounds__(256) void splitk_reduce(const float2* __restrict__ P, float2* __restrict__ C,
                                                     int64_t h, int64_t m, int64_t n, int64_t S,
                                                     const int64_t* __restrict__ offM,
                                                     const int64_t* __restrict__ offN) {
  const int64_t mn = m * n;
  const int64_t total = h * mn;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t b = idx / mn;
    const int64_t r = idx - b * mn;
    const float2* p = P + b * S * mn + r;
    float cr = 0.f, ci = 0.f;
    for (int64_t q = 0; q < S; ++q) {
      const float2 v = p[q * mn];
      cr += v.x;
      ci += v.y;
    }
    const int64_t i = r / n;
    const int64_t j = r - i * n;
    C[b * mn + (offM ? offM[i] + offN[j] : r)] = make_float2(cr, ci);
  }
}

}  // namespace

hipError_t launch_splitk_reduce(const float2* P, float2* C, int64_t h, int64_t m, int64_t n, int64_t S,
                                const int64_t* offM, const int64_t* offN, hipStream_t s) {
  const int64_t total = h * m * n;
  if (total <= 0) return hipSuccess;
  if (S <= 0) return hipErrorInvalidValue;
  int64_t grid = (total + 255) / 256;
  if (grid > 1048576) grid = 1048576;
  hipLaunchKernelGGL(splitk_reduce, dim3(grid), dim3(256), 0, s, P, C, h, m, n, S, offM, offN);
  return hipGetLastError();
}

hipError_t launch_gemm_valu(const GemmDesc& d, GemmKernel kind, Prec prec, hipStream_t s) {
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
  return hipErrorInvalidValue;
}

}  // namespace tnc
