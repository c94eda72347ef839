// FP64 cross-slice accumulation, FP64 norm, fill and conversion kernels.
//
// Slicing (paper Sec. II-C) splits the contraction into independent
// sub-networks, one per value of the sliced labels, and the answer is the
// total over them.  The per-slice results come out of the
// complex64 path; their sum is formed in FP64 in a fixed order so that a
// request's result does not depend on what else runs beside it.
#include "kernels.hpp"

namespace tnc {

namespace {

// One workgroup per output element: thread t adds s = t, t + 256, ... in
// order, then a fixed LDS tree combines the 256 partial sums.
__global__ __launch_bounds__(256) void reduce_fp64_block(const float2* root, double2* acc, int64_t hs,
                                                          int64_t R, int overwrite) {
  __shared__ double sr[256], si[256];
  const int64_t i = blockIdx.x;
  double xr = 0.0, xi = 0.0;
  for (int64_t s = threadIdx.x; s < hs; s += 256) {
    const float2 v = root[s * R + i];
    xr += static_cast<double>(v.x);
    xi += static_cast<double>(v.y);
  }
  sr[threadIdx.x] = xr;
  si[threadIdx.x] = xi;
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sr[threadIdx.x] += sr[threadIdx.x + w];
      si[threadIdx.x] += si[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double2 a = overwrite ? make_double2(0.0, 0.0) : acc[i];
    a.x += sr[0];
    a.y += si[0];
    acc[i] = a;
  }
}

// One thread per output element, s in order.
__global__ __launch_bounds__(256) void reduce_fp64_thread(const float2* root, double2* acc, int64_t hs,
                                                           int64_t R, int overwrite) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < R;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double xr = 0.0, xi = 0.0;
    for (int64_t s = 0; s < hs; ++s) {
      const float2 v = root[s * R + i];
      xr += static_cast<double>(v.x);
      xi += static_cast<double>(v.y);
    }
    double2 a = overwrite ? make_double2(0.0, 0.0) : acc[i];
    a.x += xr;
    a.y += xi;
    acc[i] = a;
  }
}

__global__ __launch_bounds__(256) void norm2_kernel(const double2* acc, int64_t R, double* out) {
  __shared__ double sm[256];
  double x = 0.0;
  for (int64_t i = threadIdx.x; i < R; i += 256) {
    const double2 v = acc[i];
    x += v.x * v.x + v.y * v.y;
  }
  sm[threadIdx.x] = x;
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint32_t* p, int64_t words) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

// Uniform values in [-1, 1) from a 32-bit integer hash of the index (the
// "lowbias32" mixer of C. Wellons' hash-prospector); stand-in operands whose
// bits toggle as real data do (all-zero operands let the MFMA pipes run
// cooler and faster than on data).
__global__ __launch_bounds__(256) void fill_hash_kernel(float* p, int64_t n, uint32_t seed) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    uint32_t x = static_cast<uint32_t>(i) ^ (static_cast<uint32_t>(i >> 32) * 0x9e3779b9u) ^ seed;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    p[i] = static_cast<float>(x >> 8) * (1.0f / 8388608.0f) - 1.0f;
  }
}

__global__ __launch_bounds__(256) void c128_to_c64_kernel(const double2* in, float2* out, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double2 v = in[i];
    out[i] = make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
  }
}

int64_t grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return g > 65536 ? 65536 : g;
}

}  // namespace

hipError_t launch_reduce_fp64(const float2* root, double2* acc, int64_t hs, int64_t R, bool overwrite,
                              hipStream_t s) {
  if (R <= 0 || hs <= 0) return hipSuccess;
  const int ow = overwrite ? 1 : 0;
  if (hs >= 64 && R <= 65536)
    hipLaunchKernelGGL(reduce_fp64_block, dim3(static_cast<unsigned>(R)), dim3(256), 0, s, root, acc, hs, R, ow);
  else
    hipLaunchKernelGGL(reduce_fp64_thread, dim3(grid_for(R)), dim3(256), 0, s, root, acc, hs, R, ow);
  return hipGetLastError();
}

hipError_t launch_norm2(const double2* acc, int64_t R, double* out, hipStream_t s) {
  hipLaunchKernelGGL(norm2_kernel, dim3(1), dim3(256), 0, s, acc, R, out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  if (bytes % 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(bytes / 4)), dim3(256), 0, s,
                     static_cast<uint32_t*>(p), bytes / 4);
  return hipGetLastError();
}

hipError_t launch_fill_hash(float* p, int64_t n, uint32_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_hash_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, seed);
  return hipGetLastError();
}

hipError_t launch_c128_to_c64(const double2* in, float2* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(c128_to_c64_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace tnc
