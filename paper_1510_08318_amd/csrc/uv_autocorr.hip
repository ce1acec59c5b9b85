// The paper's uv-plane autocorrelation removal (Sec. 4.2), once per integration.
//
// Taking the time-averaged squared image to the uv plane, subtracting the
// illumination tables' autocorrelation kernel a = sum_p n_p (K_p corr K_p)
// scaled so that its zero-spacing value equals the data's, and transforming
// back is linear in the image.  The transform of a is the summed power pattern
// Pn = sum_p n_p P_p, and the data's zero-spacing value is the image mean, so
// the whole round trip is
//     I = scale * (S - beta * Pn),   beta = sum_pix S / (N^2 a0),   a0 = a[0],
// with scale = 1/T (times the pair normalisation).  Its adjoint with respect to
// S is  dL/dS = scale * (R - <R, Pn> / (N^2 a0)): the image sensitivities shifted
// by one constant per channel.
//
// One workgroup per channel; the sums are float64, in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace moff {

namespace {

constexpr int kUvThreads = 256;

// Deterministic workgroup sum of one double per thread (valid in every thread).
__device__ __forceinline__ double block_sum(double x, double* part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
  if (lane == 0) part[wave] = x;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kUvThreads / 64; ++w) s += part[w];
  __syncthreads();
  return s;
}

}  // namespace

__global__ __launch_bounds__(kUvThreads) void uv_finalize_kernel(UvArgs a) {
  __shared__ double part[kUvThreads / 64];
  const size_t npix = static_cast<size_t>(a.N) * a.N;
  const int c = blockIdx.x;
  const float* S = a.S + static_cast<size_t>(c) * npix;
  double s = 0.0;
  for (size_t i = threadIdx.x; i < npix; i += kUvThreads) s += S[i];
  const double beta = block_sum(s, part) / (static_cast<double>(npix) * a.a0);
  float* out = a.out + static_cast<size_t>(c) * npix;
  for (size_t i = threadIdx.x; i < npix; i += kUvThreads)
    out[i] = static_cast<float>((static_cast<double>(S[i]) - beta * a.Pn[i]) * a.scale);
}

__global__ __launch_bounds__(kUvThreads) void uv_adjoint_shift_kernel(UvArgs a) {
  __shared__ double part[kUvThreads / 64];
  const size_t npix = static_cast<size_t>(a.N) * a.N;
  const int c = blockIdx.x;
  const float* R = a.S + static_cast<size_t>(c) * npix;
  double s = 0.0;
  for (size_t i = threadIdx.x; i < npix; i += kUvThreads) s += static_cast<double>(R[i]) * a.Pn[i];
  const double shift = block_sum(s, part) / (static_cast<double>(npix) * a.a0);
  float* out = a.out + static_cast<size_t>(c) * npix;
  for (size_t i = threadIdx.x; i < npix; i += kUvThreads) out[i] = static_cast<float>(static_cast<double>(R[i]) - shift);
}

hipError_t launch_uv_finalize(const UvArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(uv_finalize_kernel, dim3(a.n_chan), dim3(kUvThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_uv_adjoint_shift(const UvArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(uv_adjoint_shift_kernel, dim3(a.n_chan), dim3(kUvThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace moff
