// Device calibration: the FP32 MFMA rate and the copy bandwidth this device
// sustains, measured with a max-rate MFMA loop (independent accumulator
// chains, no memory traffic) and a 16-byte-per-lane copy.  They are the
// per-device constants of the Sec. IV-B cost model (Eq. (6)) and the
// measured ceilings kernels are compared against.
#include "kernels.hpp"

namespace tnc {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

// 8 independent chains of 16x16x4 FP32 MFMAs per wave; the sum is written
// only under a condition the inputs never meet (it keeps the loop alive).
__global__ __launch_bounds__(256) void mfma_rate_loop(float* out, int iters, float seed) {
  f4v acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f4v{0.f, 0.f, 0.f, 0.f};
  const float a = seed + threadIdx.x * 1e-7f, b = seed * 0.5f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == -1.0f) out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// 16 bytes per lane, non-temporal on both sides, one workgroup per 4096
// bytes (up to 2^20 workgroups): the fastest of the copy forms measured
// on MI355X (grid-stride loops over 1024 .. 65536 workgroups with 1 to 8
// loads in flight per lane: 4.6 .. 5.4 TB/s; this form 6.2 TB/s on 8 GiB).
__global__ __launch_bounds__(256) void copy_rate(const f4v* __restrict__ in, f4v* __restrict__ out, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    __builtin_nontemporal_store(__builtin_nontemporal_load(in + i), out + i);
}

}  // namespace

hipError_t launch_mfma_rate(float* out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(mfma_rate_loop, dim3(blocks), dim3(256), 0, s, out, iters, 1e-3f);
  return hipGetLastError();
}

hipError_t launch_copy_rate(const void* in, void* out, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 16;
  int64_t grid = (n + 255) / 256;
  if (grid > (int64_t{1} << 20)) grid = int64_t{1} << 20;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL(copy_rate, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, static_cast<const f4v*>(in),
                     static_cast<f4v*>(out), n);
  return hipGetLastError();
}

}  // namespace tnc
