// Device helpers shared by the fused kernels: sample decoding and a
// deterministic block reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace moff {

constexpr int kMaxTypesDev = 4;

__device__ __forceinline__ float2 load_sample(const void* E, size_t idx, bool ci4) {
  if (ci4) {
    // one byte: real part in the high nibble, imaginary part in the low nibble
    const int8_t b = reinterpret_cast<const int8_t*>(E)[idx];
    const int re = b >> 4;
    const int im = static_cast<int8_t>(b << 4) >> 4;
    return make_float2(static_cast<float>(re), static_cast<float>(im));
  }
  return reinterpret_cast<const float2*>(E)[idx];
}

// Deterministic block sum of four doubles per thread; result valid in thread 0..3 of `out`.
template <int NT>
__device__ __forceinline__ void block_sum4(double v[kMaxTypesDev], double* out) {
  __shared__ double part[NT / 64][kMaxTypesDev];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < kMaxTypesDev; ++p) {
    double x = v[p];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) part[wave][p] = x;
  }
  __syncthreads();
  if (threadIdx.x < kMaxTypesDev) {
    double s = 0.0;
    for (int wv = 0; wv < NT / 64; ++wv) s += part[wv][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

}  // namespace moff
