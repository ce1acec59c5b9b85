// Visibility-route (FX) imaging of one integration on the device, for
// cross-checks of the MOFF image by the paper's other method (Sec. 2: the
// time-averaged cross-products of the calibrated antenna fields, eq. cc-vis,
// gridded with each pair's power response, the cross-correlation of the two
// aperture illuminations, eq. e-field-conv, and transformed once, eq.
// dirty-image-FX, give the MOFF image; with the zero-spacing a == b terms left
// out it equals the image with the antennas' self power removed).
//
//   fx_correlate_kernel  V[c][a][b] = sum_t e_a conj(e_b), e = g E: float32
//                        products over 32-sample chunks, chunks summed in float64
//                        (complex64 samples); fx_correlate_i8_kernel: exact
//                        integer products on the matrix cores (4+4-bit samples)
//   fx_bin_kernel        H[c][pq][dy][dx] = sum of V[c][a][b] over the pairs of
//                        table types (p, q) whose footprints are offset by
//                        (dy, dx) - (L - 1) cells (plan-time CSR, fixed order)
//   fx_lag_kernel        R[c][ly][lx] = sum_pq sum_(u,v) X_pq[u][v]
//                        H[c][pq][ly - u + k_q - 1][lx - v + k_q - 1]
//   fx_row_kernel        Z[c][ly][q] = sum_lx R[c][ly][lx] w^((lx - L + 1)(q - N/2))
//   fx_col_kernel        I[c][r][q] = scale Re sum_ly w^((ly - L + 1)(r - N/2)) Z[c][ly][q]
//
// w = exp(+2 pi i / N); lags span -(L - 1) .. L - 1, so the image comes out in
// the same pixel order as the MOFF image.  Every sum runs in a fixed order
// (no atomics) and accumulates in float64; intermediate arrays are float32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fx.h"
#include "ingest.h"

namespace moff {

namespace {

constexpr int kFxTile = 32;    // antennas per side of a correlator tile
constexpr int kFxChunk = 32;   // time samples staged per step

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace

// Complex64 samples.  One workgroup per (32 x 32 antenna tile, channel); thread
// (ty, tx) owns the pairs (ty + 16 i, tx + 16 j), i, j < 2.
__global__ __launch_bounds__(256) void fx_correlate_kernel(FxArgs a) {
  __shared__ float2 ea[kFxChunk][kFxTile + 1], eb[kFxChunk][kFxTile + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int a0 = blockIdx.y * kFxTile, b0 = blockIdx.x * kFxTile, c = blockIdx.z;
  const int na = a.n_ant;
  const float2* E = reinterpret_cast<const float2*>(a.E);
  double acc[2][2][2] = {};
  for (int64_t t0 = 0; t0 < a.n_time; t0 += kFxChunk) {
    for (int k = tid; k < kFxChunk * kFxTile; k += 256) {
      const int tt = k / kFxTile, an = k % kFxTile;
      const int64_t t = t0 + tt;
      float2 va = make_float2(0.f, 0.f), vb = va;
      if (t < a.n_time) {
        const size_t base = (static_cast<size_t>(t) * a.n_chan + c) * na;
        const int ia = a0 + an, ib = b0 + an;
        if (ia < na) {
          va = E[base + ia];
          if (a.gains) va = cmul(a.gains[static_cast<size_t>(c) * na + ia], va);
        }
        if (ib < na) {
          vb = E[base + ib];
          if (a.gains) vb = cmul(a.gains[static_cast<size_t>(c) * na + ib], vb);
        }
      }
      ea[tt][an] = va;
      eb[tt][an] = vb;
    }
    __syncthreads();
    float s[2][2][2] = {};
    for (int tt = 0; tt < kFxChunk; ++tt) {
      const float2 x0 = ea[tt][ty], x1 = ea[tt][ty + 16], y0 = eb[tt][tx], y1 = eb[tt][tx + 16];
      const float2 x[2] = {x0, x1}, y[2] = {y0, y1};
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // x conj(y)
          s[i][j][0] = fmaf(x[i].x, y[j].x, fmaf(x[i].y, y[j].y, s[i][j][0]));
          s[i][j][1] = fmaf(x[i].y, y[j].x, fmaf(-x[i].x, y[j].y, s[i][j][1]));
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j][0] += s[i][j][0];
        acc[i][j][1] += s[i][j][1];
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int ia = a0 + ty + 16 * i, ib = b0 + tx + 16 * j;
      if (ia < na && ib < na)
        a.V[(static_cast<size_t>(c) * na + ia) * na + ib] =
            make_float2(static_cast<float>(acc[i][j][0]), static_cast<float>(acc[i][j][1]));
    }
}

// 4+4-bit samples: the cross-products are exact integer sums, formed on the
// matrix cores (v_mfma_i32_16x16x64_i8, int32 accumulation) from the raw
// samples; the gains are constant over the integration and are applied once,
// V_ab = g_a conj(g_b) sum_t E_a conj(E_b), in float64.  One workgroup per
// (32 x 32 antenna tile, channel), four waves of one 16 x 16 sub-tile each; per
// 64-sample step the real and imaginary parts of both antenna blocks are staged
// in LDS as int8 rows [antenna][sample] and each wave runs four products
// (re.re, im.im, im.re, re.im).  A and B take their samples in the same lane
// order, so the sum covers each sample once whatever order the instruction
// gives its contraction index; the accumulators hold D[4 (l / 16) + j][l % 16].
typedef int i32x4 __attribute__((ext_vector_type(4)));
constexpr int kI8Step = 64;                 // samples per step
constexpr int kI8Pitch = kI8Step + 16;      // LDS row bytes: 16-byte operand reads of 16 rows hit distinct banks

__global__ __launch_bounds__(256) void fx_correlate_i8_kernel(FxArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t pl[4][kFxTile][kI8Pitch];   // re A, im A, re B, im B
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int a0 = blockIdx.y * kFxTile, b0 = blockIdx.x * kFxTile, c = blockIdx.z;
  const int na = a.n_ant;
  const int8_t* E = reinterpret_cast<const int8_t*>(a.E);
  const size_t tstride = static_cast<size_t>(a.n_chan) * na;
  // staging: thread = (antenna an, group of 8 samples tg) for both blocks
  const int an = tid % kFxTile, tg = tid / kFxTile;   // tg < 8
  // this wave's sub-tile and its operand rows
  const int ah = w >> 1, bh = w & 1, l16 = lane & 15, g = lane >> 4;
  i32x4 pxx = {0, 0, 0, 0}, pyy = pxx, pyx = pxx, pxy = pxx;
  for (int64_t t0 = 0; t0 < a.n_time; t0 += kI8Step) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int ant = (blk ? b0 : a0) + an;
      uint64_t xr = 0, xi = 0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t t = t0 + 8 * tg + i;
        int8_t byte = 0;
        if (ant < na && t < a.n_time) byte = E[static_cast<size_t>(t) * tstride + static_cast<size_t>(c) * na + ant];
        const int8_t re = static_cast<int8_t>(byte >> 4);
        const int8_t im = static_cast<int8_t>(static_cast<int8_t>(byte << 4) >> 4);
        xr |= static_cast<uint64_t>(static_cast<uint8_t>(re)) << (8 * i);
        xi |= static_cast<uint64_t>(static_cast<uint8_t>(im)) << (8 * i);
      }
      *reinterpret_cast<uint64_t*>(&pl[2 * blk][an][8 * tg]) = xr;
      *reinterpret_cast<uint64_t*>(&pl[2 * blk + 1][an][8 * tg]) = xi;
    }
    __syncthreads();
    const i32x4 ar = *reinterpret_cast<const i32x4*>(&pl[0][16 * ah + l16][16 * g]);
    const i32x4 ai = *reinterpret_cast<const i32x4*>(&pl[1][16 * ah + l16][16 * g]);
    const i32x4 br = *reinterpret_cast<const i32x4*>(&pl[2][16 * bh + l16][16 * g]);
    const i32x4 bi = *reinterpret_cast<const i32x4*>(&pl[3][16 * bh + l16][16 * g]);
    pxx = __builtin_amdgcn_mfma_i32_16x16x64_i8(ar, br, pxx, 0, 0, 0);
    pyy = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai, bi, pyy, 0, 0, 0);
    pyx = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai, br, pyx, 0, 0, 0);
    pxy = __builtin_amdgcn_mfma_i32_16x16x64_i8(ar, bi, pxy, 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ia = a0 + 16 * ah + 4 * g + j, ib = b0 + 16 * bh + l16;
    if (ia >= na || ib >= na) continue;
    // E_a conj(E_b) = (xa xb + ya yb) + i (ya xb - xa yb)
    const double vr = static_cast<double>(pxx[j]) + pyy[j], vi = static_cast<double>(pyx[j]) - pxy[j];
    double zr = vr, zi = vi;
    if (a.gains) {
      const float2 ga = a.gains[static_cast<size_t>(c) * na + ia], gb = a.gains[static_cast<size_t>(c) * na + ib];
      // g_a conj(g_b)
      const double gr = static_cast<double>(ga.x) * gb.x + static_cast<double>(ga.y) * gb.y;
      const double gi = static_cast<double>(ga.y) * gb.x - static_cast<double>(ga.x) * gb.y;
      zr = gr * vr - gi * vi;
      zi = gr * vi + gi * vr;
    }
    a.V[(static_cast<size_t>(c) * na + ia) * na + ib] = make_float2(static_cast<float>(zr), static_cast<float>(zi));
  }
}

// One thread per (channel, type pair, offset cell).
__global__ __launch_bounds__(256) void fx_bin_kernel(FxArgs a) {
  const size_t cells = static_cast<size_t>(a.n_types) * a.n_types * a.NL * a.NL;
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= cells) return;
  const int c = blockIdx.y;
  const float2* V = a.V + static_cast<size_t>(c) * a.n_ant * a.n_ant;
  double x = 0.0, y = 0.0;
  for (int k = a.pair_ptr[i]; k < a.pair_ptr[i + 1]; ++k) {
    const float2 v = V[a.pair_ab[k]];
    x += v.x;
    y += v.y;
  }
  a.H[static_cast<size_t>(c) * cells + i] = make_float2(static_cast<float>(x), static_cast<float>(y));
}

// One thread per (channel, lag cell).
__global__ __launch_bounds__(256) void fx_lag_kernel(FxArgs a) {
  const int NL = a.NL;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NL * NL) return;
  const int c = blockIdx.y, ly = i / NL, lx = i % NL;
  const size_t plane = static_cast<size_t>(NL) * NL;
  double x = 0.0, y = 0.0;
  for (int p = 0; p < a.n_types; ++p)
    for (int q = 0; q < a.n_types; ++q) {
      const int tp = p * a.n_types + q;
      const int kb = a.ktype_k[q], side = a.ktype_k[p] + kb - 1;
      const float2* H = a.H + (static_cast<size_t>(c) * a.n_types * a.n_types + tp) * plane;
      const float2* X = a.xcorr + static_cast<size_t>(tp) * a.xs * a.xs;
      for (int u = 0; u < side; ++u) {
        const int hy = ly - u + kb - 1;
        if (hy < 0 || hy >= NL) continue;
        for (int v = 0; v < side; ++v) {
          const int hx = lx - v + kb - 1;
          if (hx < 0 || hx >= NL) continue;
          const float2 h = H[static_cast<size_t>(hy) * NL + hx], w = X[u * a.xs + v];
          x += static_cast<double>(w.x) * h.x - static_cast<double>(w.y) * h.y;
          y += static_cast<double>(w.x) * h.y + static_cast<double>(w.y) * h.x;
        }
      }
    }
  a.R[static_cast<size_t>(c) * plane + i] = make_float2(static_cast<float>(x), static_cast<float>(y));
}

// One workgroup of N threads per (lag row ly, channel); thread q.
__global__ __launch_bounds__(256) void fx_row_kernel(FxArgs a) {
  extern __shared__ float2 fx_lds[];
  float2* row = fx_lds;            // [NL]
  float2* tw = fx_lds + a.NL;      // [N]
  const int N = a.N, NL = a.NL, ly = blockIdx.x, c = blockIdx.y, q = threadIdx.x;
  const float2* Rrow = a.R + (static_cast<size_t>(c) * NL + ly) * NL;
  for (int k = q; k < NL; k += N) row[k] = Rrow[k];
  tw[q] = a.tw[q];
  __syncthreads();
  const int s = q - N / 2;
  double x = 0.0, y = 0.0;
  for (int lx = 0; lx < NL; ++lx) {
    const float2 w = tw[((lx - (a.L - 1)) * s) & (N - 1)], r = row[lx];
    x += static_cast<double>(r.x) * w.x - static_cast<double>(r.y) * w.y;
    y += static_cast<double>(r.x) * w.y + static_cast<double>(r.y) * w.x;
  }
  a.Z[(static_cast<size_t>(c) * NL + ly) * N + q] = make_float2(static_cast<float>(x), static_cast<float>(y));
}

// One workgroup of N threads per (block of kFxRows image rows, channel);
// thread q reads each Z[ly][q] once for all the block's rows.
constexpr int kFxRows = 8;

__global__ __launch_bounds__(256) void fx_col_kernel(FxArgs a) {
  const int N = a.N, NL = a.NL, r0 = blockIdx.x * kFxRows, c = blockIdx.y, q = threadIdx.x;
  const float2* Z = a.Z + static_cast<size_t>(c) * NL * N;
  double x[kFxRows] = {};
  for (int ly = 0; ly < NL; ++ly) {
    const float2 z = Z[static_cast<size_t>(ly) * N + q];
    const int d = ly - (a.L - 1);
#pragma unroll
    for (int k = 0; k < kFxRows; ++k) {
      const float2 w = a.tw[(d * (r0 + k - N / 2)) & (N - 1)];
      x[k] += static_cast<double>(w.x) * z.x - static_cast<double>(w.y) * z.y;
    }
  }
#pragma unroll
  for (int k = 0; k < kFxRows; ++k) a.out[(static_cast<size_t>(c) * N + r0 + k) * N + q] = static_cast<float>(x[k] * a.scale);
}

hipError_t launch_fx(const FxArgs& a, bool ci4, hipStream_t st) {
  if (a.n_ant < 1 || a.n_chan < 1 || a.n_chan > 65535 || a.N < 8 || a.N > 256 || a.NL != 2 * a.L - 1 ||
      a.n_types < 1 || a.n_types > kMaxTypesDev)
    return hipErrorInvalidValue;
  const unsigned tiles = static_cast<unsigned>((a.n_ant + kFxTile - 1) / kFxTile);
  const dim3 g1(tiles, tiles, static_cast<unsigned>(a.n_chan));
  if (ci4)
    hipLaunchKernelGGL(fx_correlate_i8_kernel, g1, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(fx_correlate_kernel, g1, dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t cells = static_cast<size_t>(a.n_types) * a.n_types * a.NL * a.NL;
  hipLaunchKernelGGL(fx_bin_kernel, dim3(static_cast<unsigned>((cells + 255) / 256), a.n_chan), dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned lag_blocks = static_cast<unsigned>((a.NL * a.NL + 255) / 256);
  hipLaunchKernelGGL(fx_lag_kernel, dim3(lag_blocks, a.n_chan), dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds = sizeof(float2) * (a.NL + a.N);
  hipLaunchKernelGGL(fx_row_kernel, dim3(a.NL, a.n_chan), dim3(a.N), lds, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(fx_col_kernel, dim3(a.N / kFxRows, a.n_chan), dim3(a.N), 0, st, a);
  return hipGetLastError();
}

}  // namespace moff
