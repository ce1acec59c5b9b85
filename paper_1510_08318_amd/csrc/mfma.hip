// Reduced-precision MOFF frame transform on the gfx950 matrix cores.
//
// For grids of 64 and 128 the padded 2-D DFT of Sec. 3 is computed as two
// dense complex matrix products (Sec. 6.1 counts the transform as the dominant
// cost; at these sizes the contraction is small enough to run as plain matrix
// products):
//
//   row stage     Z[iy][q] = sum_ix Eg[iy][ix] W[ix][q],  W[ix][q] = exp(+2 pi i ix (q - N/2) / N) / (N/2)
//   column stage  Y[r][q]  = sum_iy V[r][iy] Z[iy][q],    V[r][iy] = exp(+2 pi i iy (r - N/2) / N)
//
// over the L = N/2 nonzero rows and columns of the zero-padded grid, so the
// outputs come out directly in image pixel order (index N/2 is the phase
// centre).  Each complex product is one real product of doubled contraction
// length: [Re x | Im x] times [[Re w, Im w], [-Im w, Re w]] gives [Re, Im] of
// x w.  Operands are binary16 or bfloat16 (Eg rounded once when gridded, Z once
// between the stages, W and V once from float64 phase factors); every product
// accumulates in float32 (v_mfma_f32_32x32x16_{f16,bf16}).
//
// One workgroup (2 waves at N = 64, 4 at N = 128) owns one (channel, time
// slice) and loops over its frames; per frame:
//   1. ingest + calibration: e = g E into LDS (float32), self power in float64
//      (the next frame's samples are loaded during this frame's matrix work);
//   2. gather-gridding: each lane walks its balanced slice of the cell-keyed
//      program (no atomics) and stores finished cells as 16-bit values;
//   3. row stage: each wave owns a 32-column block of Z (and part of its
//      rows), with that block's W operands held in registers for the whole
//      launch and Eg read from LDS; Z is written to LDS transposed
//      (column-major), the layout the column stage reads;
//   4. column stage: the same wave owns the same-numbered 32-row block of Y
//      (and part of its columns), with that block's V operands in registers,
//      and accumulates |Y|^2 in registers.
// Registers are held to 256 per lane so that two workgroups share each CU:
// their frames drift out of step, and one workgroup's matrix work overlaps the
// other's gathering and LDS traffic (8-wave workgroups, whose waves meet at the
// same barriers, were 15 % slower at N = 128).
// After the last frame the accumulators go through the same epilogue modes as
// the float32 fused kernel (per-slice partial, running sum, final image).
//
// MFMA operand layout (32x32x16, checked on the device): lane l supplies
// A[l % 32][8 (l / 32) + i] and B[8 (l / 32) + i][l % 32], i < 8, and receives
// D[8 (j / 4) + 4 (l / 32) + j % 4][l % 32] in accumulator j < 16.
//
// LDS rows are 2L + 8 sixteen-bit elements long: the 16-byte operand reads of
// eight consecutive rows then fall in eight different 16-byte bank groups.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dft.h"
#include "ingest.h"
#include "kernels.h"

namespace moff {

namespace {

template <class H>
struct Vec {
  typedef H v8 __attribute__((ext_vector_type(8)));
  typedef H v4 __attribute__((ext_vector_type(4)));
};
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <class H>
__device__ __forceinline__ f32x16 mfma32(typename Vec<H>::v8 a, typename Vec<H>::v8 b, f32x16 c);

template <>
__device__ __forceinline__ f32x16 mfma32<_Float16>(Vec<_Float16>::v8 a, Vec<_Float16>::v8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f32x16 mfma32<__bf16>(Vec<__bf16>::v8 a, Vec<__bf16>::v8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

template <int N>
struct MfmaShape {
  static constexpr int L = N / 2;
  static constexpr int NW = mfma_waves(N); // waves per workgroup
  static constexpr int NT = NW * 64;
  static constexpr int KS = L / 8;         // 16-deep steps over the doubled contraction 2L
  static constexpr int NB = N / 32;        // output blocks: row-stage column blocks = column-stage row blocks
  static constexpr int WPB = NW / NB;      // waves sharing one output block
  static constexpr int RBW = L / 32 / WPB; // row stage: 32-row blocks per wave
  static constexpr int CBW = NB / WPB;     // column stage: 32-column blocks per wave
  static_assert(NW % NB == 0 && RBW >= 1 && CBW >= 1, "wave split must tile both stages");
  static constexpr int PITCH = 2 * L + 8;  // LDS row length, 16-bit elements
  static constexpr int EG = L * PITCH;     // Eg [L][PITCH]: real parts at ix, imaginary at L + ix
  static constexpr int ZT = N * PITCH;     // Zt [N][PITCH]: Zt[q][iy] = Re Z, Zt[q][L + iy] = Im Z
};

}  // namespace

size_t mfma_lds_bytes(int N, int n_taps, int n_ant, int prog_len, bool prog_in_lds) {
  const MfmaLayout m = mfma_layout(N, n_taps, n_ant);
  const size_t prog = prog_in_lds ? sizeof(GatherEntry) * static_cast<size_t>(prog_len) * (mfma_waves(N) * 64) : 0;
  return static_cast<size_t>(m.prog) + prog;
}

bool mfma_prog_fits_lds(int N, int n_taps, int n_ant, int prog_len) {
  return mfma_lds_bytes(N, n_taps, n_ant, prog_len, true) <= kMfmaProgLdsLimit;
}

template <int N, class H, bool CI4>
__global__ __launch_bounds__((MfmaShape<N>::NT)) __attribute__((amdgpu_waves_per_eu(2)))
void mfma_kernel(MfmaArgs a) {
  using S = MfmaShape<N>;
  using V8 = typename Vec<H>::v8;
  using V4 = typename Vec<H>::v4;
  constexpr int NT = S::NT, L = S::L, KS = S::KS, PITCH = S::PITCH;
  extern __shared__ uint4 lds_mfma[];
  __shared__ double Atot[kMaxTypesDev];
  char* lds = reinterpret_cast<char*>(lds_mfma);
  const MfmaLayout lay = mfma_layout(N, a.n_taps, a.n_ant);
  float2* e = reinterpret_cast<float2*>(lds + lay.e);   // [n_ant + 1], last slot stays zero
  float2* K = reinterpret_cast<float2*>(lds + lay.k);   // [n_taps]
  H* Eg = reinterpret_cast<H*>(lds + lay.eg);
  H* Zt = reinterpret_cast<H*>(lds + lay.zt);
  float2* gl = reinterpret_cast<float2*>(lds + lay.gl); // [n_ant]
  int* ty = reinterpret_cast<int*>(lds + lay.ty);       // [n_ant]
  // gather program [prog_len][NT], copied into LDS when it fits
  GatherEntry* lprog = reinterpret_cast<GatherEntry*>(lds + lay.prog);

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // wave w owns output block blk (its row-stage columns and column-stage rows)
  // and part sub of that block's other dimension
  const int blk = w / S::WPB, sub = w % S::WPB;
  const int item = blockIdx.x;
  if (item >= a.n_chan * a.slices) return;
  const int c = item % a.n_chan;
  const int slice = item / a.n_chan;

  // phase-factor operands of this wave, resident for the whole launch
  V8 w_re[KS], w_im[KS], v_re[KS], v_im[KS];
  {
    const V8* src = reinterpret_cast<const V8*>(a.dft);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      w_re[ks] = src[(((0 * S::NB + blk) * KS + ks) * 2 + 0) * 64 + lane];
      w_im[ks] = src[(((0 * S::NB + blk) * KS + ks) * 2 + 1) * 64 + lane];
      v_re[ks] = src[(((1 * S::NB + blk) * KS + ks) * 2 + 0) * 64 + lane];
      v_im[ks] = src[(((1 * S::NB + blk) * KS + ks) * 2 + 1) * 64 + lane];
    }
  }

  // clear the aperture grid once: cells without antennas are never written
  for (int i = tid; i < S::EG * 2 / 16; i += NT) reinterpret_cast<uint4*>(Eg)[i] = make_uint4(0u, 0u, 0u, 0u);
  for (int i = tid; i < a.n_taps; i += NT) K[i] = a.ktab[i];
  for (int i = tid; i < a.n_ant; i += NT) {
    ty[i] = a.ant_type[i];
    gl[i] = a.gains ? a.gains[static_cast<size_t>(c) * a.n_ant + i] : make_float2(1.f, 0.f);
  }
  if (tid == 0) e[a.n_ant] = make_float2(0.f, 0.f);
  if (a.prog_in_lds)
    for (int i = tid; i < a.prog_len * NT; i += NT) lprog[i] = a.prog[i];

  const int64_t T = a.n_time;
  const int64_t t0 = slice * T / a.slices, t1 = (slice + 1) * T / a.slices;
  const size_t frame_stride = static_cast<size_t>(a.n_chan) * a.n_ant;
  const GatherEntry* prog = (a.prog_in_lds ? lprog : a.prog) + tid;

  // Raw samples of the next frame are loaded into registers before the row
  // stage and used after the column stage, so the HBM latency is hidden behind
  // the matrix work.  The first kPrefetch * NT antennas keep their self power
  // in a register (one slot each); antennas beyond that are loaded when used.
  // Per-thread self-power sums are float32 (this path's error budget is set by
  // its 16-bit operands); threads are combined in float64.
  constexpr int kPrefetch = N == 128 ? 1 : 4;
  float2 raw[kPrefetch];
  float pws[kPrefetch];
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) pws[j] = 0.f;
  auto load_raw = [&](int64_t t) {
    const size_t base = static_cast<size_t>(t) * frame_stride + static_cast<size_t>(c) * a.n_ant;
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int i = tid + j * NT;
      if (i < a.n_ant) raw[j] = load_sample(a.E, base + i, CI4);
    }
  };
  float pwt[kMaxTypesDev] = {0.f, 0.f, 0.f, 0.f};
  auto calibrate = [&](int i, float2 x) {
    const float2 v = c_mul(gl[i], x);
    e[i] = v;
    const float p = fmaf(v.x, v.x, v.y * v.y);
    const int tp = ty[i];
#pragma unroll
    for (int q = 0; q < kMaxTypesDev; ++q) pwt[q] += (tp == q) ? p : 0.f;
  };
  auto ingest = [&](int64_t t) {
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int i = tid + j * NT;
      if (i < a.n_ant) {
        const float2 v = c_mul(gl[i], raw[j]);
        e[i] = v;
        pws[j] += fmaf(v.x, v.x, v.y * v.y);
      }
    }
    const size_t base = static_cast<size_t>(t) * frame_stride + static_cast<size_t>(c) * a.n_ant;
    for (int i = tid + kPrefetch * NT; i < a.n_ant; i += NT) calibrate(i, load_sample(a.E, base + i, CI4));
  };

  float acc[S::CBW][16];
#pragma unroll
  for (int cb = 0; cb < S::CBW; ++cb)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[cb][j] = 0.f;
  const int row = lane & 31, half = lane >> 5;
  __syncthreads();   // tables in LDS
  if (t0 < t1) load_raw(t0);
  for (int64_t t = t0; t < t1; ++t) {
    // 1. ingest + calibration (samples loaded during the previous frame); e[] was
    //    last read by the previous frame's gather, finished before its row stage
    ingest(t);
    __syncthreads();

    // 2. gather-gridding into 16-bit cells
    {
      float2 g = make_float2(0.f, 0.f);
      // entry: x = byte offsets of e[ant] (low half) and K[tap] (high half),
      // y = byte address of the finished cell's real part, or 0
      auto step = [&](GatherEntry en) {
        const float2 ev = *reinterpret_cast<const float2*>(lds + (en.x & 0xFFFFu));
        const float2 kv = *reinterpret_cast<const float2*>(lds + (en.x >> 16));
        g.x = fmaf(ev.x, kv.x, fmaf(-ev.y, kv.y, g.x));
        g.y = fmaf(ev.x, kv.y, fmaf(ev.y, kv.x, g.y));
        if (en.y != 0u) {
          H* cell = reinterpret_cast<H*>(lds + en.y);
          cell[0] = static_cast<H>(g.x);
          cell[L] = static_cast<H>(g.y);
          g = make_float2(0.f, 0.f);
        }
      };
      int k = 0;
      for (; k + 4 <= a.prog_len; k += 4) {
        GatherEntry en[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) en[i] = prog[static_cast<size_t>(k + i) * NT];
#pragma unroll
        for (int i = 0; i < 4; ++i) step(en[i]);
      }
      for (; k < a.prog_len; ++k) step(prog[static_cast<size_t>(k) * NT]);
    }
    __syncthreads();
    if (t + 1 < t1) load_raw(t + 1);

    // 3. row stage: Z = Eg W for the 32 output columns of block blk
#pragma unroll
    for (int i_rb = 0; i_rb < S::RBW; ++i_rb) {
      const int rb = sub * S::RBW + i_rb;
      f32x16 zr = {}, zi = {};
      const H* arow = Eg + (32 * rb + row) * PITCH + 8 * half;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const V8 av = *reinterpret_cast<const V8*>(arow + 16 * ks);
        zr = mfma32<H>(av, w_re[ks], zr);
        zi = mfma32<H>(av, w_im[ks], zi);
      }
      // lane holds rows iy = 32 rb + 8 g + 4 half + (0..3) of column q = 32 blk + row
      H* zcol = Zt + (32 * blk + row) * PITCH + 32 * rb + 4 * half;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        V4 vr, vi;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          vr[i] = static_cast<H>(zr[4 * g + i]);
          vi[i] = static_cast<H>(zi[4 * g + i]);
        }
        *reinterpret_cast<V4*>(zcol + 8 * g) = vr;
        *reinterpret_cast<V4*>(zcol + 8 * g + L) = vi;
      }
    }
    __syncthreads();

    // 4. column stage: Y = V Z for the 32 output rows of block blk, |Y|^2 accumulated
#pragma unroll
    for (int i_cb = 0; i_cb < S::CBW; ++i_cb) {
      const int cb = sub * S::CBW + i_cb;
      f32x16 yr = {}, yi = {};
      const H* bcol = Zt + (32 * cb + row) * PITCH + 8 * half;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const V8 bv = *reinterpret_cast<const V8*>(bcol + 16 * ks);
        yr = mfma32<H>(v_re[ks], bv, yr);
        yi = mfma32<H>(v_im[ks], bv, yi);
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[i_cb][j] = fmaf(yr[j], yr[j], fmaf(yi[j], yi[j], acc[i_cb][j]));
    }
  }

  double pw[kMaxTypesDev];
#pragma unroll
  for (int q = 0; q < kMaxTypesDev; ++q) pw[q] = pwt[q];
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) {
    const int i = tid + j * NT;
    if (i < a.n_ant) {
      const int tp = ty[i];
#pragma unroll
      for (int q = 0; q < kMaxTypesDev; ++q) pw[q] += (tp == q) ? static_cast<double>(pws[j]) : 0.0;
    }
  }
  block_sum4<NT>(pw, Atot);

  // epilogue: the row stage carried a factor 1 / L, so |Y|^2 is scaled back by L^2 (exact)
  const size_t img_stride = static_cast<size_t>(N) * N;
  constexpr float kBack = static_cast<float>(L) * static_cast<float>(L);
#pragma unroll
  for (int i_cb = 0; i_cb < S::CBW; ++i_cb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int r = 32 * blk + 8 * (j / 4) + 4 * half + (j % 4);
      const int q = 32 * (sub * S::CBW + i_cb) + row;
      const size_t pix = static_cast<size_t>(r) * N + q;
      const float s = acc[i_cb][j] * kBack;
      if (a.mode == kModePartial) {
        a.out[(static_cast<size_t>(slice) * a.n_chan + c) * img_stride + pix] = s;
      } else if (a.mode == kModeAccum) {
        a.out[static_cast<size_t>(c) * img_stride + pix] += s;
      } else {
        double v = s;
        if (a.subtract)
          for (int p = 0; p < a.n_types; ++p) v -= Atot[p] * a.Pp[p * img_stride + pix];
        a.out[static_cast<size_t>(c) * img_stride + pix] = static_cast<float>(v * a.scale);
      }
    }
  if (tid < a.n_types) {
    if (a.mode == kModePartial) {
      a.outA[(static_cast<size_t>(slice) * a.n_chan + c) * a.n_types + tid] = Atot[tid];
    } else if (a.mode == kModeAccum) {
      a.outA[static_cast<size_t>(c) * a.n_types + tid] += Atot[tid];
    }
  }
}

namespace {

template <int N, class H, bool CI4>
hipError_t launch_mfma_t(const MfmaArgs& a, int grid, hipStream_t st) {
  const size_t lds = mfma_lds_bytes(N, a.n_taps, a.n_ant, a.prog_len, a.prog_in_lds != 0);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mfma_kernel<N, H, CI4>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((mfma_kernel<N, H, CI4>), dim3(grid), dim3(MfmaShape<N>::NT), lds, st, a);
  return hipGetLastError();
}

template <int N, class H, bool CI4>
int blocks_t(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&mfma_kernel<N, H, CI4>),
                                                   MfmaShape<N>::NT, lds) != hipSuccess)
    return 1;
  return n;
}

}  // namespace

int mfma_threads(int N) { return N == 64 ? MfmaShape<64>::NT : MfmaShape<128>::NT; }

hipError_t launch_mfma(const MfmaArgs& a, int N, int prec, bool ci4, int grid, hipStream_t st) {
  if (N == 64) {
    if (prec == 2) return ci4 ? launch_mfma_t<64, __bf16, true>(a, grid, st) : launch_mfma_t<64, __bf16, false>(a, grid, st);
    return ci4 ? launch_mfma_t<64, _Float16, true>(a, grid, st) : launch_mfma_t<64, _Float16, false>(a, grid, st);
  }
  if (N == 128) {
    if (prec == 2)
      return ci4 ? launch_mfma_t<128, __bf16, true>(a, grid, st) : launch_mfma_t<128, __bf16, false>(a, grid, st);
    return ci4 ? launch_mfma_t<128, _Float16, true>(a, grid, st) : launch_mfma_t<128, _Float16, false>(a, grid, st);
  }
  return hipErrorInvalidValue;
}

int mfma_blocks_per_cu(int N, int prec, bool ci4, size_t lds) {
  if (N == 64) {
    if (prec == 2) return ci4 ? blocks_t<64, __bf16, true>(lds) : blocks_t<64, __bf16, false>(lds);
    return ci4 ? blocks_t<64, _Float16, true>(lds) : blocks_t<64, _Float16, false>(lds);
  }
  if (prec == 2) return ci4 ? blocks_t<128, __bf16, true>(lds) : blocks_t<128, __bf16, false>(lds);
  return ci4 ? blocks_t<128, _Float16, true>(lds) : blocks_t<128, _Float16, false>(lds);
}

}  // namespace moff
