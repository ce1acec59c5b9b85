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

// Issue priority by progress through a work item's frames [t0, t1), for
// kernels whose workgroups share a CU: 3 in the first half of the frames, 2
// in the next fourth, 1 in the next eighth and 0 in the last eighth.
// Otherwise a CU's oldest waves issue first, its workgroups advance unevenly,
// and the first to finish leaves the CU short of waves for the others'
// remaining frames.  A workgroup that has fallen behind across a boundary
// outranks the ones ahead until it catches up, so the spread left at the end
// is what builds up within the last, shortest segment.  Only the order in
// which ready waves issue changes, never a result.  frame(t) runs at the top
// of frame t; every call is wave-uniform.  Compiled out (Enabled false) for
// shapes that never share a CU.
template <bool Enabled>
struct ProgressPrio {
  bool on;
  int level;   // boundaries crossed
  int64_t next, step;
  __device__ ProgressPrio(bool on_, int64_t t0, int64_t t1)
      : on(Enabled && on_), level(0), next(t0 + (t1 - t0) / 2), step((t1 - t0) / 4) {
    if constexpr (Enabled)
      if (on) __builtin_amdgcn_s_setprio(3);
  }
  __device__ __forceinline__ void frame(int64_t t) {
    if constexpr (Enabled) {
      if (on && t == next && level < 3) {
        ++level;
        next += step;
        step /= 2;
        if (level == 1) __builtin_amdgcn_s_setprio(2);
        else if (level == 2) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
      }
    }
  }
  __device__ __forceinline__ void done() const {
    if constexpr (Enabled)
      if (on) __builtin_amdgcn_s_setprio(0);
  }
};

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
