// gfx950 kernels of the MOFF imaging path.
//
//   fused_kernel      ingest + calibration + gather-gridding + padded 2-D DFT +
//                     |.|^2 + time accumulation (+ self-power removal) for all
//                     frames of one (column class, channel, time slice); one
//                     launch covers every channel (Sec. 2 MOFF imaging equation,
//                     Sec. 3 implementation steps, Sec. 4.2 autocorrelations).
//   reduce_kernel     fixed-order reduction of per-slice partial sums, then
//                     self-power removal and averaging (or accumulation).
//   grid_kernel, self_power_kernel, fft2_kernel, detect_kernel, finalize_kernel
//                     the same steps one at a time through HBM (staged path).
//
// Every output element has exactly one writer and every sum is taken in a
// fixed order, so results are bitwise reproducible.  The only global atomics
// are the no-return float64 adds of blocked accumulation, each into a running
// sum that one lane alone writes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "frame.h"
#include "ingest.h"
#include "kernels.h"


namespace moff {

namespace {

// exp(+2 pi i k / SX) for SX dividing 4, exact.
__device__ __forceinline__ float2 quarter_rot(float2 v, int k, int SX) {
  const int q = ((k * (4 / SX)) % 4 + 4) % 4;
  return q == 0 ? v : q == 1 ? c_mul_i(v) : q == 2 ? c_neg(v) : c_mul_mi(v);
}

// Gather-gridding of one frame into the folded grid: each lane walks its slice
// of the cell-keyed program, multiplies the calibrated antenna field by the
// tap weight, and stores each finished cell sum.  Every folded cell is written.
// A lane's cells are consecutive in row-major order from its first cell, so
// an entry carries only the antenna slot, the weight index and a "cell
// complete" bit (4 bytes, four per 16-byte load), and the k-th store of a lane
// goes to cell cell0 + k.  With real weights (RW) each entry's weight comes
// with it from the program (progw), which halves the LDS reads -- the
// gather's limit -- and the multiply-adds; otherwise it is looked up in the
// LDS weight table W.  With destination-carrying entries (DST: real weights,
// and a grid that leaves room for one workgroup per CU, where no other
// workgroup hides the per-cell store branch) an entry carries its cell's LDS
// element and a first-of-cell flag instead, and every entry stores its cell's
// running sum; the cell's last entry stores the final one.  The program sits
// in global memory (L2-resident: it is the same for every frame) and is read
// in whole batches of B entries, then the rest four at a time, so that no
// entry past the program's end is executed and a batch has no trip-count
// branches.  The samples, weights and grid are disjoint LDS arrays
// (restrict), and the LDS values of S entries are read before any of their
// stores: a conditional store starts a new basic block, and reads placed after
// it would each wait for a full LDS round trip.
template <int NT, int B, int S, int NZR, int ZP, bool RW, bool DST>
__device__ __forceinline__ void gather_frame(const uint4* __restrict__ prog, const float4* __restrict__ progw,
                                             int prog_len, int cell0, const float2* __restrict__ e,
                                             const float2* __restrict__ W, float2* __restrict__ G) {
  static_assert(B % 4 == 0 && B % S == 0, "batches hold whole 16-byte loads and LDS sub-batches");
  static_assert(RW || !DST, "destination-carrying entries come with their weights");
  static_assert((NZR & (NZR - 1)) == 0, "folded rows are a power of two long");
  float2 acc = make_float2(0.f, 0.f);
  uint32_t cell = static_cast<uint32_t>(cell0);   // unsigned: the row split below is a shift
  // one batch of BB entries from 16-byte word k0 on, in sub-batches of SS
  auto batch = [&](int k0, auto bc, auto sc) {
    constexpr int BB = decltype(bc)::value, SS = decltype(sc)::value;
    uint32_t ent[BB];
    float wt[RW ? BB : 1];
#pragma unroll
    for (int j = 0; j < BB / 4; ++j) {
      const size_t at = static_cast<size_t>(k0 + j) * NT;
      const uint4 q = prog[at];
      ent[4 * j] = q.x;
      ent[4 * j + 1] = q.y;
      ent[4 * j + 2] = q.z;
      ent[4 * j + 3] = q.w;
      if constexpr (RW) {
        const float4 qw = progw[at];
        wt[4 * j] = qw.x;
        wt[4 * j + 1] = qw.y;
        wt[4 * j + 2] = qw.z;
        wt[4 * j + 3] = qw.w;
      }
    }
#pragma unroll
    for (int s0 = 0; s0 < BB; s0 += SS) {
      float2 ev[SS], wv[RW ? 1 : SS];
#pragma unroll
      for (int i = 0; i < SS; ++i) {
        ev[i] = e[ent[s0 + i] & 0xFFFu];
        if constexpr (!RW) wv[i] = W[(ent[s0 + i] >> 12) & 0x7FFu];
      }
#pragma unroll
      for (int i = 0; i < SS; ++i) {
        if constexpr (DST) {
          // every entry stores its cell's running sum: no branch per cell
          const bool first = ent[s0 + i] & kFirstBit;
          acc.x = fmaf(ev[i].x, wt[s0 + i], first ? 0.f : acc.x);
          acc.y = fmaf(ev[i].y, wt[s0 + i], first ? 0.f : acc.y);
          G[(ent[s0 + i] >> 12) & 0xFFFFu] = acc;
          continue;
        }
        if constexpr (RW) {
          acc.x = fmaf(ev[i].x, wt[s0 + i], acc.x);
          acc.y = fmaf(ev[i].y, wt[s0 + i], acc.y);
        } else {
          acc.x = fmaf(ev[i].x, wv[i].x, fmaf(-ev[i].y, wv[i].y, acc.x));
          acc.y = fmaf(ev[i].x, wv[i].y, fmaf(ev[i].y, wv[i].x, acc.y));
        }
        if (ent[s0 + i] & kStoreBit) {
          G[cell + (cell / NZR) * (ZP - NZR)] = acc;   // folded cell (a, n') at a ZP + n'
          ++cell;
          acc = make_float2(0.f, 0.f);
        }
      }
    }
  };
  // whole batches of B, then the rest (a multiple of 4 entries) four at a time
  const int len4 = prog_len / 4;
  int k0 = 0;
  for (; k0 + B / 4 <= len4; k0 += B / 4)
    batch(k0, std::integral_constant<int, B>{}, std::integral_constant<int, S>{});
  for (; k0 < len4; ++k0) batch(k0, std::integral_constant<int, 4>{}, std::integral_constant<int, (S < 4 ? S : 4)>{});
}

// The gather in the entry form the plan provides (uniform branches).
template <int NT, int B, int S, int NZR, int ZP>
__device__ __forceinline__ void gather_frame_any(const uint4* __restrict__ prog, const float4* __restrict__ progw,
                                                 int prog_len, int cell0, bool dst_entries,
                                                 const float2* __restrict__ e, const float2* __restrict__ W,
                                                 float2* __restrict__ G) {
  if (progw && dst_entries)
    gather_frame<NT, B, S, NZR, ZP, true, true>(prog, progw, prog_len, cell0, e, W, G);
  else if (progw)
    gather_frame<NT, B, S, NZR, ZP, true, false>(prog, progw, prog_len, cell0, e, W, G);
  else
    gather_frame<NT, B, S, NZR, ZP, false, false>(prog, progw, prog_len, cell0, e, W, G);
}

// Entries per batch of program reads (B) and per LDS sub-batch (S): short
// batches measured fastest at both N = 128 and 256 (8 and 4 against 12–16
// and 4–8: 2.21 against 2.24 ms at the LWA shape, 23.7 against 24.5 ms at
// the HERA shape).
constexpr int kGatherBatch = 8;
constexpr int kGatherSub = 4;

}  // namespace

// ---------------------------------------------------------------------------
// fused kernel
// ---------------------------------------------------------------------------

// Waves per SIMD the fused kernel's registers are sized for: at N = 128,
// shape variant 0 fits four (128 registers), which several workgroups per CU
// need to hide one another's gather latency.
template <int N, int V>
constexpr int fused_waves_per_simd() {
  return (N == 128 && V == 0) ? 4 : 1;
}

// Whether workgroups of a shape can share a CU (its LDS leaves room for a
// second): at N = 256 shape variant 1 the 132 KB folded grid does not.
constexpr bool shares_cu(int N, int V) { return !(N == 256 && V == 1); }

// One work item of the fused kernel: column class W (a compile-time constant,
// so the row stage's fold factors are constant rotations), channel c and a
// slice of time samples.  ONE: every lane ingests at most one antenna
// (n_ant <= NT), so a lane's self power is one float64 sum, given its type
// after the frame loop, instead of one running sum per antenna type (8 fewer
// registers held through the loop: at the HERA shape 1 spilled register
// instead of 24).  The sums are the same either way.
template <int N, int V, bool CI4, int W, bool ONE>
__device__ __forceinline__ void fused_item(const FusedArgs& a, float2* lds, double* Atot, int c, int slice,
                                           int item) {
  using C = FT<N, V>;
  constexpr int NT = C::NT;
  const int tid = threadIdx.x;

  float2* G = lds;                          // [L][P], row pitch P = M + 1
  float2* twr = G + C::GRID;                // [PR * QR]
  float2* twc = twr + C::TWR;               // [PC * QC]
  float2* Wt = twc + C::TWC;                // [n_weights]
  float2* gl = Wt + a.n_weights;            // [n_ant] gains of the current channel
  float2* e = gl + a.n_ant;                 // [n_ant + 1], last slot stays zero
  int* ty = reinterpret_cast<int*>(e + a.n_ant + 1);  // [n_ant]

  for (int i = tid; i < a.n_ant; i += NT) ty[i] = a.ant_type[i];
  if (tid == 0) e[a.n_ant] = make_float2(0.f, 0.f);
  const int64_t T = a.n_time;
  const size_t frame_stride = static_cast<size_t>(a.n_chan) * a.n_ant;
  const size_t img_stride = static_cast<size_t>(N) * N;

  build_twiddles<N, V>(a.tw, W, twr, twc);
  for (int i = tid; i < a.n_weights; i += NT) Wt[i] = a.weights[static_cast<size_t>(W) * a.n_weights + i];
  for (int i = tid; i < a.n_ant; i += NT)
    gl[i] = a.gains ? a.gains[static_cast<size_t>(c) * a.n_ant + i] : make_float2(1.f, 0.f);

  const int64_t t0 = slice * T / a.slices, t1 = (slice + 1) * T / a.slices;
  const uint4* prog = a.prog + static_cast<size_t>(W) * (a.prog_len / 4) * NT + tid;
  const float4* progw = a.progw ? a.progw + static_cast<size_t>(W) * (a.prog_len / 4) * NT + tid : nullptr;
  const int cell0 = a.cell0[W * NT + tid];

  float acc[C::NACC];
#pragma unroll
  for (int i = 0; i < C::NACC; ++i) acc[i] = 0.f;
  double pw[kMaxTypesDev] = {0.0, 0.0, 0.0, 0.0};
  double pw1 = 0.0;   // ONE: the lane's antenna's self power
  // float64 running sums of this workgroup's pixels (blocked accumulation),
  // laid out [item][acc index][lane]: a uniform base per accumulator index
  // plus the lane's offset, so no per-lane address stays live in the loop
  double* run64 = a.acc64 ? a.acc64 + static_cast<size_t>(item) * C::NACC * NT : nullptr;
  bool flushed = false;
  int in_block = 0;

  // (at the LWA shape with one round of four workgroups per CU: 2.17 ms with
  // the progress priority, 2.42 ms without)
  ProgressPrio<shares_cu(N, V)> prio(a.progress_prio != 0, t0, t1);
  __syncthreads();
  for (int64_t t = t0; t < t1; ++t) {
    prio.frame(t);
    // ingest + calibration: e = g * E, and the self power of each antenna type
    const size_t base = static_cast<size_t>(t) * frame_stride + static_cast<size_t>(c) * a.n_ant;
    auto take = [&](int i, float2 raw_v) {
      const float2 v = c_mul(gl[i], raw_v);
      e[i] = v;
      const double p = static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y;
      if constexpr (ONE) {
        pw1 += p;
      } else {
        const int tp = ty[i];
#pragma unroll
        for (int q = 0; q < kMaxTypesDev; ++q) pw[q] += (tp == q) ? p : 0.0;
      }
    };
    if constexpr (ONE) {
      if (tid < a.n_ant) take(tid, load_sample(a.E, base + tid, CI4));
    } else {
      for (int i = tid; i < a.n_ant; i += NT) take(i, load_sample(a.E, base + i, CI4));
    }
    __syncthreads();
    gather_frame_any<NT, kGatherBatch, kGatherSub, C::NZR, C::P>(prog, progw, a.prog_len, cell0, a.dst_entries, e,
                                                                 Wt, G);
    // With wave-owned rows each wave has gridded exactly the rows it
    // transforms next, so its own LDS order suffices (a uniform branch).
    if (a.wave_rows) wave_sync();
    else __syncthreads();
    row_stage_w<N, V, W>(G, twr);
    __syncthreads();
    col_stage<N, V>(G, twc, [&](int idx, int, int, float2 v) { acc[idx] = fmaf(v.x, v.x, fmaf(v.y, v.y, acc[idx])); });
    // blocked accumulation: fold the block's float32 sums into float64
    if (a.acc64 && ++in_block == kBlockFrames && t + 1 < t1) {   // uniform branch
      // An opaque zero defined here keeps the compiler from hoisting the
      // flush's addresses out of the time loop (they would hold 2 NACC
      // registers for the whole loop).
      int zero;
      asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
      double* blk = run64 + zero + tid;
      // The first block is stored, later ones added (no-return float64 adds:
      // each address has this one lane as its only writer, so the order of
      // additions is fixed).
      if (!flushed) {
#pragma unroll
        for (int idx = 0; idx < C::NACC; ++idx) blk[idx * NT] = static_cast<double>(acc[idx]);
      } else {
#pragma unroll
        for (int idx = 0; idx < C::NACC; ++idx) unsafeAtomicAdd(blk + idx * NT, static_cast<double>(acc[idx]));
      }
#pragma unroll
      for (int idx = 0; idx < C::NACC; ++idx) acc[idx] = 0.f;
      flushed = true;
      in_block = 0;
    }
  }

  prio.done();
  if constexpr (ONE) {
    if (tid < a.n_ant) {
      const int tp = ty[tid];
#pragma unroll
      for (int q = 0; q < kMaxTypesDev; ++q) pw[q] = (tp == q) ? pw1 : 0.0;
    }
  }
  // (its barriers also end every wave's use of the folded grid)
  block_sum4<NT>(pw, Atot);

  // The transform runs on the transposed aperture (the host plan's programs):
  // its folded axis m is the image row, r = SX m + W, and its column-stage
  // output index is the image column, so this workgroup owns whole image rows.
  // A lane's pixels are scattered over those rows, so finished float values
  // are staged in LDS (the grid's space, [M][N + 4] floats) and written out
  // row by row; only the in-place float64 update of accumulate mode writes
  // per pixel.  Within a staged row, groups of four pixels are permuted by an
  // XOR with the row's swizzle (a multiple of 4), which spreads one store
  // instruction's 16 rows over the LDS banks.
  float* stage = reinterpret_cast<float*>(lds);
  static_assert(C::M * N * sizeof(float) <= C::GRID * sizeof(float2), "staging must fit in the grid");
  auto swz = [](int col) { return (col << 2) & (N - 4); };
#pragma unroll
  for (int idx = 0; idx < C::NACC; ++idx) {
    int r, col;
    acc_pixel<N, V>(idx, r, col);
    if (C::CGUARD && col >= C::M) continue;
    const int pr = (C::SX * col + W + N / 2) & (N - 1), pq = (r + N / 2) & (N - 1);
    const size_t pix = static_cast<size_t>(pr) * N + pq;
    // (read at device scope: the adds were performed in L2)
    const double sum = static_cast<double>(acc[idx]) +
                       (flushed ? __hip_atomic_load(run64 + idx * NT + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : 0.0);
    if (a.mode == kModePartial) {
      stage[col * N + (pq ^ swz(col))] = static_cast<float>(sum);
    } else if (a.mode == kModeAccum) {
      float& o = a.out[static_cast<size_t>(c) * img_stride + pix];
      o = static_cast<float>(static_cast<double>(o) + sum);
    } else {
      double v = sum;
      if (a.subtract)
        for (int p = 0; p < a.n_types; ++p) v -= Atot[p] * a.Pp[p * img_stride + pix];
      stage[col * N + (pq ^ swz(col))] = static_cast<float>(v * a.scale);
    }
  }
  if (a.mode != kModeAccum) {
    __syncthreads();
    float* dst = a.out + (a.mode == kModePartial ? (static_cast<size_t>(slice) * a.n_chan + c) : static_cast<size_t>(c)) *
                             img_stride;
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
      for (int i = tid; i < C::M * (N / 4); i += NT) {
        const int col = i / (N / 4), q = 4 * (i % (N / 4));
        const int pr = (C::SX * col + W + N / 2) & (N - 1);
        *reinterpret_cast<float4*>(dst + static_cast<size_t>(pr) * N + q) =
            *reinterpret_cast<const float4*>(stage + col * N + (q ^ swz(col)));
      }
    } else {
      for (int i = tid; i < C::M * N; i += NT) {
        const int col = i / N, q = i % N;
        dst[static_cast<size_t>((C::SX * col + W + N / 2) & (N - 1)) * N + q] = stage[col * N + (q ^ swz(col))];
      }
    }
  }
  if (W == 0 && tid < a.n_types) {
    if (a.mode == kModePartial) {
      a.outA[(static_cast<size_t>(slice) * a.n_chan + c) * a.n_types + tid] = Atot[tid];
    } else if (a.mode == kModeAccum) {
      a.outA[static_cast<size_t>(c) * a.n_types + tid] += Atot[tid];
    }
  }
}

// One work item (output class w, channel c, time slice) per workgroup.  (A
// persistent loop over items makes the compiler keep far more registers live
// -- 127 -> 256 VGPRs at N = 64 -- so launches are instead sized in whole
// rounds of resident workgroups by the autotuner.)  Workgroups are dealt to
// the XCDs round-robin by index, so the decode gives each XCD a contiguous
// range of (channel, slice) indices, with the SX classes of one index kXcds
// apart: the classes share their samples in that XCD's L2, and neighbouring
// channels share the 128-byte lines their samples straddle.  The grid pads the
// (channel, slice) count to a multiple of kXcds.
template <int N, int V, bool CI4, bool ONE>
__global__ __launch_bounds__((FT<N, V>::NT)) __attribute__((amdgpu_waves_per_eu(fused_waves_per_simd<N, V>())))
void fused_kernel(FusedArgs a) {
  using C = FT<N, V>;
  extern __shared__ float2 lds[];
  __shared__ double Atot[kMaxTypesDev];
  const int b = blockIdx.x, k = b / kXcds;
  const int per_xcd = gridDim.x / (kXcds * C::SX);            // (channel, slice) indices per XCD
  const int w = k % C::SX;
  const int cs = (b % kXcds) * per_xcd + k / C::SX;           // channel-slice index
  if (cs >= a.n_chan * a.slices) return;
  const int c = cs % a.n_chan, slice = cs / a.n_chan;
  const int item = cs * C::SX + w;
  static_for<0, C::SX>([&](auto wc) {
    constexpr int W = decltype(wc)::value;
    if (w == W) fused_item<N, V, CI4, W, ONE>(a, lds, Atot, c, slice, item);
  });
}

// ---------------------------------------------------------------------------
// fused gain adjoint
// ---------------------------------------------------------------------------

// One work item of the fused gain adjoint: output class W (compile-time, as in
// the forward kernel), channel c and a slice of time samples.  Per frame, in
// LDS: ingest, gather-gridding with the forward program, the row stage, the
// column round trip (forward column DFT, each pixel times its sensitivity,
// adjoint column DFT), the row-stage adjoint and the degridding of this lane's
// antennas.  The sensitivities come from memory per column job (Rl, laid out
// by adjoint_sensitivity_kernel so that each lane's values are contiguous),
// not from registers held for the whole launch.
template <int N, int V, bool CI4, int W>
__device__ __forceinline__ void adjoint_item(const AdjFusedArgs& a, float2* lds, int c, int slice) {
  using C = FT<N, V>;
  constexpr int NT = C::NT;
  const int tid = threadIdx.x;

  float2* G = lds;                          // [L][P], row pitch P = M + 1
  float2* twr = G + C::GRID;                // [PR * QR]
  float2* twc = twr + C::TWR;               // [PC * QC]
  float2* Wt = twc + C::TWC;                // [n_weights]
  float2* gl = Wt + a.n_weights;            // [n_ant] gains of the current channel
  float2* e = gl + a.n_ant;                 // [n_ant + 1], last slot stays zero

  build_twiddles<N, V>(a.tw, W, twr, twc);
  for (int i = tid; i < a.n_weights; i += NT) Wt[i] = a.weights[static_cast<size_t>(W) * a.n_weights + i];
  for (int i = tid; i < a.n_ant; i += NT)
    gl[i] = a.gains ? a.gains[static_cast<size_t>(c) * a.n_ant + i] : make_float2(1.f, 0.f);
  if (tid == 0) e[a.n_ant] = make_float2(0.f, 0.f);

  // this lane's sensitivities, in the layout of adjoint_sensitivity_kernel
  const float* Rlane = a.Rl + (static_cast<size_t>(c) * C::SX + W) * C::NACC * NT;

  // this lane's antennas for the degridding (their descriptors and samples are
  // read again at the degridding, not held through the transforms)
  double2 D[kAdjSlots];
#pragma unroll
  for (int s = 0; s < kAdjSlots; ++s) D[s] = make_double2(0.0, 0.0);
  const uint2* slots = reinterpret_cast<const uint2*>(a.slots) + static_cast<size_t>(tid) * kAdjSlots;

  const int64_t T = a.n_time;
  const int64_t t0 = slice * T / a.slices, t1 = (slice + 1) * T / a.slices;
  const size_t frame_stride = static_cast<size_t>(a.n_chan) * a.n_ant;
  const uint4* prog = a.prog + static_cast<size_t>(W) * (a.prog_len / 4) * NT + tid;
  const float4* progw = a.progw ? a.progw + static_cast<size_t>(W) * (a.prog_len / 4) * NT + tid : nullptr;
  const int cell0 = a.cell0[W * NT + tid];

  ProgressPrio<shares_cu(N, V)> prio(a.progress_prio != 0, t0, t1);
  __syncthreads();
  for (int64_t t = t0; t < t1; ++t) {
    prio.frame(t);
    const size_t base = static_cast<size_t>(t) * frame_stride + static_cast<size_t>(c) * a.n_ant;
    for (int i = tid; i < a.n_ant; i += NT) e[i] = c_mul(gl[i], load_sample(a.E, base + i, CI4));
    __syncthreads();
    gather_frame_any<NT, kGatherBatch, kGatherSub, C::NZR, C::P>(prog, progw, a.prog_len, cell0, a.dst_entries, e,
                                                                 Wt, G);
    if (a.wave_rows) wave_sync();   // (wave-owned rows: as in the forward kernel)
    else __syncthreads();
    row_stage_w<N, V, W>(G, twr);
    __syncthreads();
    col_stage_roundtrip<N, V>(G, twc, [&](int cs, int s, int jb, float (&rr)[C::QC]) {
      const int idx0 = ((cs * 2 + s) * C::JB + jb) * C::QC;
      if constexpr (C::QC % 4 == 0) {
#pragma unroll
        for (int k = 0; k < C::QC / 4; ++k) {
          const float4 q = reinterpret_cast<const float4*>(Rlane)[static_cast<size_t>(idx0 / 4 + k) * NT + tid];
          rr[4 * k] = q.x;
          rr[4 * k + 1] = q.y;
          rr[4 * k + 2] = q.z;
          rr[4 * k + 3] = q.w;
        }
      } else {
#pragma unroll
        for (int k = 0; k < C::QC; ++k) rr[k] = Rlane[static_cast<size_t>(idx0 + k) * NT + tid];
      }
    });
    __syncthreads();
    // this lane's antennas and their raw samples load while the row-stage adjoint runs
    uint2 sl[kAdjSlots];
    float2 Er[kAdjSlots];
#pragma unroll
    for (int s = 0; s < kAdjSlots; ++s) {
      sl[s] = slots[s];
      const uint32_t ant = sl[s].x & 0xFFFu;
      Er[s] = ant != kAdjEmpty ? load_sample(a.E, base + ant, CI4) : make_float2(0.f, 0.f);
    }
    row_stage_adjoint_w<N, V, W>(G, twr);
    __syncthreads();
    // degridding: d = sum over the footprint of conj(weight) G', then D += conj(E) d
#pragma unroll
    for (int s = 0; s < kAdjSlots; ++s) {
      const uint32_t ant = sl[s].x & 0xFFFu;
      if (ant == kAdjEmpty) continue;
      const int off = (sl[s].x >> 12) & 0xFFFu, k = (sl[s].x >> 24) & 0xFu;
      const int ix0 = sl[s].y & 0xFFFFu, iy0 = sl[s].y >> 16;
      float dx = 0.f, dy = 0.f;
      // transposed aperture: folded-grid row ix, folded axis along y
      for (int v = 0; v < k; ++v) {
        const float2* Grow = G + (ix0 + v) * C::P;
        for (int u = 0; u < k; ++u) {
          const int iy = iy0 + u;
          const int j = iy / C::M, n = iy - j * C::M;
          const float2 g = Grow[n];
          const float2 wt = Wt[j * a.n_taps + off + u * k + v];
          dx = fmaf(g.x, wt.x, fmaf(g.y, wt.y, dx));
          dy = fmaf(g.y, wt.x, fmaf(-g.x, wt.y, dy));
        }
      }
      D[s].x += static_cast<double>(Er[s].x) * dx + static_cast<double>(Er[s].y) * dy;
      D[s].y += static_cast<double>(Er[s].x) * dy - static_cast<double>(Er[s].y) * dx;
    }
  }
  prio.done();
#pragma unroll
  for (int s = 0; s < kAdjSlots; ++s) {
    const uint32_t ant = slots[s].x & 0xFFFu;
    if (ant == kAdjEmpty) continue;
    a.Dp[(static_cast<size_t>(slice * C::SX + W) * a.n_chan + c) * a.n_ant + ant] = D[s];
  }
}

// WPS: the least number of waves per SIMD the registers are sized for (1: as
// many registers as the kernel wants).  Built where it fits and chosen by the
// plan's autotuner together with the shape variant.
template <int N, int V, bool CI4, int WPS>
__global__ __launch_bounds__((FT<N, V>::NT)) __attribute__((amdgpu_waves_per_eu(WPS)))
void adjoint_fused_kernel(AdjFusedArgs a) {
  using C = FT<N, V>;
  extern __shared__ float2 lds[];
  const int item = blockIdx.x;
  if (item >= C::SX * a.n_chan * a.slices) return;
  const int w = item % C::SX;
  const int c = (item / C::SX) % a.n_chan;
  const int slice = item / (C::SX * a.n_chan);
  static_for<0, C::SX>([&](auto wc) {
    constexpr int W = decltype(wc)::value;
    if (w == W) adjoint_item<N, V, CI4, W>(a, lds, c, slice);
  });
}

// Sensitivities dL/dI [C][N][N] rearranged per (channel, output class) so that
// each lane of the fused adjoint reads its column-job values contiguously:
// Rl[c][w] holds NACC x NT floats, accumulator index idx of thread tid at
// ((idx / 4) NT + tid) 4 + idx % 4 when QC is a multiple of 4 (one 16-byte
// load per 4 values), else at idx NT + tid.  The pixel of (w, tid, idx) is the
// one the fused kernels' column stage produces there (transposed aperture:
// image row SX col + w, image column r); columns past M read 0.
template <int N, int V>
__global__ __launch_bounds__(256) void adjoint_sensitivity_kernel(const float* R, int n_chan, float* Rl) {
  using C = FT<N, V>;
  const size_t per_class = static_cast<size_t>(C::NACC) * C::NT;
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= per_class * C::SX * n_chan) return;
  const size_t cw = i / per_class, k = i % per_class;
  const int c = static_cast<int>(cw / C::SX), w = static_cast<int>(cw % C::SX);
  int idx, tid;
  if constexpr (C::QC % 4 == 0) {
    idx = static_cast<int>((k / (4 * C::NT)) * 4 + k % 4);
    tid = static_cast<int>((k / 4) % C::NT);
  } else {
    idx = static_cast<int>(k / C::NT);
    tid = static_cast<int>(k % C::NT);
  }
  int r, col;
  acc_pixel_of<N, V>(tid, idx, r, col);
  float v = 0.f;
  if (!(C::CGUARD && col >= C::M)) {
    const int pr = (C::SX * col + w + N / 2) & (N - 1), pq = (r + N / 2) & (N - 1);
    v = R[(static_cast<size_t>(c) * N + pr) * N + pq];
  }
  Rl[i] = v;
}

// One thread per (channel, antenna): Q = sum_t |E|^2 in float64.
template <bool CI4>
__global__ __launch_bounds__(256) void antenna_power_kernel(const void* E, int64_t n_time, int n_chan, int n_ant,
                                                            double* Q) {
  const int c = blockIdx.y;
  const int ant = blockIdx.x * 256 + threadIdx.x;
  if (ant >= n_ant) return;
  double q = 0.0;
  for (int64_t t = 0; t < n_time; ++t) {
    const float2 v = load_sample(E, (static_cast<size_t>(t) * n_chan + c) * n_ant + ant, CI4);
    q += static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y;
  }
  Q[static_cast<size_t>(c) * n_ant + ant] = q;
}

// D = sum of the per-(slice, class) partial sums, in order.
__global__ __launch_bounds__(256) void adjoint_reduce_kernel(const double2* Dp, int parts, size_t n, double2* D) {
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  double x = 0.0, y = 0.0;
  for (int k = 0; k < parts; ++k) {
    x += Dp[static_cast<size_t>(k) * n + i].x;
    y += Dp[static_cast<size_t>(k) * n + i].y;
  }
  D[i] = make_double2(x, y);
}

// Sum per-slice partials (pixel order) in slice order, four pixels per thread
// (N^2 is a multiple of 4, and each slice's loads are independent so they are
// issued four slices at a time); then remove self power and average
// (MODE_FINAL) or add into the caller's running sums (MODE_ACCUM).
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
  const size_t npix = static_cast<size_t>(a.N) * a.N;
  const size_t i = (static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (i >= npix * a.n_chan) return;
  const size_t c = i / npix, pix = i % npix;
  const size_t stride4 = static_cast<size_t>(a.n_chan) * npix / 4;   // one slice, in float4
  const float4* src = reinterpret_cast<const float4*>(a.S_part) + i / 4;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  auto add = [&](float4 v) {
    s[0] += v.x;
    s[1] += v.y;
    s[2] += v.z;
    s[3] += v.w;
  };
  int sl = 0;
  for (; sl + 4 <= a.slices; sl += 4) {
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = src[static_cast<size_t>(sl + k) * stride4];
#pragma unroll
    for (int k = 0; k < 4; ++k) add(v[k]);
  }
  for (; sl < a.slices; ++sl) add(src[static_cast<size_t>(sl) * stride4]);
  double A[kMaxTypesDev] = {0.0, 0.0, 0.0, 0.0};
  for (int p = 0; p < a.n_types; ++p)
    for (int q = 0; q < a.slices; ++q) A[p] += a.A_part[(static_cast<size_t>(q) * a.n_chan + c) * a.n_types + p];
  float r[4];
  if (a.final_image) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double v = s[k];
      if (a.subtract)
        for (int p = 0; p < a.n_types; ++p) v -= A[p] * a.Pp[p * npix + pix + k];
      r[k] = static_cast<float>(v * a.scale);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = a.out[i + k] + static_cast<float>(s[k]);
    if (pix == 0)
      for (int p = 0; p < a.n_types; ++p) a.outA[c * a.n_types + p] += A[p];
  }
  if ((reinterpret_cast<uintptr_t>(a.out + i) & 15) == 0) {
    *reinterpret_cast<float4*>(a.out + i) = make_float4(r[0], r[1], r[2], r[3]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) a.out[i + k] = r[k];
  }
}

// ---------------------------------------------------------------------------
// staged kernels
// ---------------------------------------------------------------------------

// One workgroup per frame: calibrate into LDS, then every aperture cell sums
// its CSR row (antenna-ascending) and writes Eg.
template <bool CI4>
__global__ __launch_bounds__(256) void grid_kernel(GridArgs a) {
  extern __shared__ float2 lds[];
  float2* e = lds;               // [n_ant]
  float2* K = e + a.n_ant;       // [n_taps]
  const int64_t f = blockIdx.x;  // frame = t * n_chan + c
  const int c = static_cast<int>(f % a.n_chan);
  const size_t base = static_cast<size_t>(f) * a.n_ant;
  for (int i = threadIdx.x; i < a.n_ant; i += 256) {
    const float2 g = a.gains ? a.gains[static_cast<size_t>(c) * a.n_ant + i] : make_float2(1.f, 0.f);
    e[i] = c_mul(g, load_sample(a.E, base + i, CI4));
  }
  for (int i = threadIdx.x; i < a.n_taps; i += 256) K[i] = a.ktab[i];
  __syncthreads();
  const int ncell = a.L * a.L;
  float2* out = a.Eg + static_cast<size_t>(f) * ncell;
  for (int cell = threadIdx.x; cell < ncell; cell += 256) {
    float2 s = make_float2(0.f, 0.f);
    for (int k = a.csr_ptr[cell]; k < a.csr_ptr[cell + 1]; ++k) {
      const float2 ev = e[a.csr_ant[k]], kv = K[a.csr_tap[k]];
      s.x = fmaf(ev.x, kv.x, fmaf(-ev.y, kv.y, s.x));
      s.y = fmaf(ev.x, kv.y, fmaf(ev.y, kv.x, s.y));
    }
    out[cell] = s;
  }
}

// One workgroup per channel: A[c][p] += sum_t sum_{a of type p} |g E|^2.
template <bool CI4>
__global__ __launch_bounds__(256) void self_power_kernel(GridArgs a) {
  __shared__ double tot[kMaxTypesDev];
  const int c = blockIdx.x;
  double pw[kMaxTypesDev] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < a.n_ant; i += 256) {
    const float2 g = a.gains ? a.gains[static_cast<size_t>(c) * a.n_ant + i] : make_float2(1.f, 0.f);
    const int tp = a.ant_type[i];
    double s = 0.0;
    for (int64_t t = 0; t < a.n_time; ++t) {
      const float2 v = c_mul(g, load_sample(a.E, (static_cast<size_t>(t) * a.n_chan + c) * a.n_ant + i, CI4));
      s += static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y;
    }
#pragma unroll
    for (int q = 0; q < kMaxTypesDev; ++q) pw[q] += (tp == q) ? s : 0.0;
  }
  block_sum4<256>(pw, tot);
  if (threadIdx.x < a.n_types) a.A[static_cast<size_t>(c) * a.n_types + threadIdx.x] += tot[threadIdx.x];
}

// One workgroup per (column class, frame): load and fold the aperture grid,
// transform, store the complex image field in pixel order.
template <int N>
__global__ __launch_bounds__((FT<N, 0>::NT)) void fft2_kernel(Fft2Args a) {
  using C = FT<N, 0>;
  extern __shared__ float2 lds[];
  float2* G = lds;
  float2* twr = G + C::GRID;
  float2* twc = twr + C::TWR;
  const int w = blockIdx.x % C::SX;
  const int64_t f = blockIdx.x / C::SX;
  build_twiddles<N, 0>(a.tw, w, twr, twc);
  float2 fin[C::PRNZ];
  fold_factors<N, 0>(a.tw, w, fin);
  const float2* src = a.Eg + static_cast<size_t>(f) * C::L * C::L;
  for (int cell = threadIdx.x; cell < C::L * C::NZR; cell += C::NT) {
    const int iy = cell / C::NZR, n = cell % C::NZR;
    float2 v = make_float2(0.f, 0.f);
    for (int j = 0; j * C::M + n < C::L; ++j) {
      const float2 x = quarter_rot(src[iy * C::L + n + j * C::M], j * w, C::SX);
      v = c_add(v, x);
    }
    G[iy * C::P + n] = v;
  }
  __syncthreads();
  row_stage<N, 0>(G, twr, fin);
  __syncthreads();
  float2* dst = a.Y + static_cast<size_t>(f) * N * N;
  col_stage<N, 0>(G, twc, [&](int, int r, int col, float2 v) {
    const int q = C::SX * col + w;
    dst[((r + N / 2) & (N - 1)) * N + ((q + N / 2) & (N - 1))] = v;
  });
}

// One thread per (channel, pixel): S += sum_t |Y|^2.
__global__ __launch_bounds__(256) void detect_kernel(DetectArgs a) {
  const size_t npix = static_cast<size_t>(a.N) * a.N;
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= npix * a.n_chan) return;
  const size_t stride = npix * a.n_chan;
  float s = 0.f;
  for (int64_t t = 0; t < a.n_time; ++t) {
    const float2 v = a.Y[static_cast<size_t>(t) * stride + i];
    s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
  }
  a.S[i] += s;
}

// image = (S - sum_p A_p P_p) * scale
__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a) {
  const size_t npix = static_cast<size_t>(a.N) * a.N;
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= npix * a.n_chan) return;
  const size_t c = i / npix, pix = i % npix;
  double v = a.S[i];
  if (a.subtract)
    for (int p = 0; p < a.n_types; ++p) v -= a.A[c * a.n_types + p] * a.Pp[p * npix + pix];
  a.out[i] = static_cast<float>(v * a.scale);
}

// ---------------------------------------------------------------------------
// gain gradient (adjoint of the path)
// ---------------------------------------------------------------------------

// One workgroup per (column class, frame): Y' = R * Y on the class's pixels,
// adjoint column and row passes, store the folded adjoint grid.
template <int N>
__global__ __launch_bounds__((FT<N, 0>::NT)) void adjoint_fft2_kernel(AdjFftArgs a) {
  using C = FT<N, 0>;
  extern __shared__ float2 lds[];
  float2* G = lds;
  float2* twr = G + C::GRID;
  float2* twc = twr + C::TWR;
  const int w = blockIdx.x % C::SX;
  const int64_t f = blockIdx.x / C::SX;
  const int c = static_cast<int>(f % a.n_chan);
  build_twiddles<N, 0>(a.tw, w, twr, twc);
  float2 fin[C::PRNZ];
  fold_factors<N, 0>(a.tw, w, fin);
  __syncthreads();
  const float2* Y = a.Y + static_cast<size_t>(f) * N * N;
  const float* R = a.R + static_cast<size_t>(c) * N * N;
  col_stage_adjoint<N, 0>(G, twc, [&](int, int r, int col) -> float2 {
    const int q = C::SX * col + w;
    const size_t pix = static_cast<size_t>((r + N / 2) & (N - 1)) * N + ((q + N / 2) & (N - 1));
    const float2 y = Y[pix];
    const float rr = R[pix];
    return make_float2(y.x * rr, y.y * rr);
  });
  __syncthreads();
  row_stage_adjoint<N, 0>(G, twr, fin);
  __syncthreads();
  float2* out = a.Gp + (static_cast<size_t>(f) * C::SX + w) * C::L * C::NZR;
  for (int cell = threadIdx.x; cell < C::L * C::NZR; cell += C::NT) {
    const int iy = cell / C::NZR, n = cell % C::NZR;
    out[cell] = G[iy * C::P + n];
  }
}

// One thread per (channel, antenna): d_t = sum over footprint taps and column
// classes of conj(weight) * G'_t, then D += conj(E_t) d_t and Q += |E_t|^2 in
// float64 over the chunk's time samples.
template <bool CI4>
__global__ __launch_bounds__(256) void degrid_kernel(DegridArgs a) {
  const int c = blockIdx.y;
  const int ant = blockIdx.x * 256 + threadIdx.x;
  if (ant >= a.n_ant) return;
  const int p = a.ant_type[ant];
  const int k = a.ktype_k[p], off = a.ktype_off[p];
  const int ix0 = a.ant_cells[2 * ant], iy0 = a.ant_cells[2 * ant + 1];
  const int nw = a.NJ * a.n_taps;
  double Dx = 0.0, Dy = 0.0, Q = 0.0;
  for (int64_t t = 0; t < a.n_time; ++t) {
    const int64_t f = t * a.n_chan + c;
    float dx = 0.f, dy = 0.f;
    for (int w = 0; w < a.SX; ++w) {
      const float2* Gw = a.Gp + (static_cast<size_t>(f) * a.SX + w) * a.L * a.NZR;
      const float2* Ww = a.weights + static_cast<size_t>(w) * nw;
      for (int u = 0; u < k; ++u) {
        const float2* Grow = Gw + static_cast<size_t>(iy0 + u) * a.NZR;
        for (int v = 0; v < k; ++v) {
          const int ix = ix0 + v;
          const int j = ix / a.M, n = ix - j * a.M;
          const float2 g = Grow[n];
          const float2 wt = Ww[j * a.n_taps + off + u * k + v];
          dx = fmaf(g.x, wt.x, fmaf(g.y, wt.y, dx));     // g * conj(wt)
          dy = fmaf(g.y, wt.x, fmaf(-g.x, wt.y, dy));
        }
      }
    }
    const float2 e = load_sample(a.E, (static_cast<size_t>(t) * a.n_chan + c) * a.n_ant + ant, CI4);
    Dx += static_cast<double>(e.x) * dx + static_cast<double>(e.y) * dy;   // conj(e) * d
    Dy += static_cast<double>(e.x) * dy - static_cast<double>(e.y) * dx;
    Q += static_cast<double>(e.x) * e.x + static_cast<double>(e.y) * e.y;
  }
  const size_t i = static_cast<size_t>(c) * a.n_ant + ant;
  a.D[i] = make_double2(a.D[i].x + Dx, a.D[i].y + Dy);
  a.Q[i] += Q;
}

// One workgroup per channel: rho_p = sum_pix R P_p, then
// grad = scale (D - rho_{p(a)} g Q).
__global__ __launch_bounds__(256) void grad_final_kernel(GradFinalArgs a) {
  __shared__ double rho[kMaxTypesDev];
  const int c = blockIdx.x;
  const size_t npix = static_cast<size_t>(a.N) * a.N;
  double part[kMaxTypesDev] = {0.0, 0.0, 0.0, 0.0};
  if (a.subtract) {
    const float* R = a.R + static_cast<size_t>(c) * npix;
    for (size_t i = threadIdx.x; i < npix; i += 256) {
      const double r = R[i];
      for (int p = 0; p < a.n_types; ++p) part[p] += r * a.Pp[p * npix + i];
    }
  }
  block_sum4<256>(part, rho);
  for (int ant = threadIdx.x; ant < a.n_ant; ant += 256) {
    const size_t i = static_cast<size_t>(c) * a.n_ant + ant;
    double gx = a.D[i].x, gy = a.D[i].y;
    if (a.subtract) {
      const float2 g = a.gains ? a.gains[i] : make_float2(1.f, 0.f);
      const double s = rho[a.ant_type[ant]] * a.Q[i];
      gx -= s * g.x;
      gy -= s * g.y;
    }
    a.grad[i] = make_float2(static_cast<float>(gx * a.scale), static_cast<float>(gy * a.scale));
  }
}

// Fill with zeros (a kernel rather than a memset node, so captured graphs replay it safely).
__global__ __launch_bounds__(256) void zero_kernel(uint32_t* p, size_t n) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += static_cast<size_t>(gridDim.x) * 256)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

size_t fused_lds_bytes(int N, int V, int n_weights, int n_ant) {
  const FrameShape S = frame_shape(N, V);
  const int M = N / S.SX, L = N / 2;
  return sizeof(float2) * (static_cast<size_t>(L) * grid_pitch(M) + S.PR * S.QR + S.PC * S.QC + n_weights + n_ant +
                           n_ant + 1) +
         sizeof(int) * n_ant;
}

namespace {

template <int N, int V, bool CI4>
const void* fused_symbol(bool one) {
  return one ? reinterpret_cast<const void*>(fused_kernel<N, V, CI4, true>)
             : reinterpret_cast<const void*>(fused_kernel<N, V, CI4, false>);
}

template <int N, int V>
const void* fused_symbol_v(bool ci4, bool one) {
  if constexpr (frame_shape(N, V).N == N)
    return ci4 ? fused_symbol<N, V, true>(one) : fused_symbol<N, V, false>(one);
  else
    return nullptr;
}

// one: the variant for at most one antenna per lane (n_ant <= threads)
const void* fused_kernel_symbol(int N, int V, bool ci4, bool one) {
  auto pick = [&](auto nc) -> const void* {
    constexpr int NN = decltype(nc)::value;
    return V == 0 ? fused_symbol_v<NN, 0>(ci4, one) : V == 1 ? fused_symbol_v<NN, 1>(ci4, one) : nullptr;
  };
  switch (N) {
    case 8: return pick(std::integral_constant<int, 8>{});
    case 16: return pick(std::integral_constant<int, 16>{});
    case 32: return pick(std::integral_constant<int, 32>{});
    case 64: return pick(std::integral_constant<int, 64>{});
    case 128: return pick(std::integral_constant<int, 128>{});
    case 256: return pick(std::integral_constant<int, 256>{});
    default: return nullptr;
  }
}

template <int N>
hipError_t launch_fft2_t(const Fft2Args& a, int64_t n_frames, hipStream_t st) {
  const FrameShape S = frame_shape(N);
  const size_t lds = sizeof(float2) * (static_cast<size_t>(N / 2) * grid_pitch(N / S.SX) + N / S.SX + N);
  auto k = fft2_kernel<N>;
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(n_frames * S.SX)), dim3(S.NT), lds, st, a);  // caller keeps it < 2^31
  return hipGetLastError();
}

unsigned blocks_for(size_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

hipError_t launch_fused(const FusedArgs& a, int N, int V, bool ci4, int grid, hipStream_t st) {
  const FrameShape S = frame_shape(N, V);
  const void* k = fused_kernel_symbol(N, V, ci4, a.n_ant <= S.NT);
  if (!k) return hipErrorInvalidValue;
  // the kernel's decode assumes SX classes times a whole number of XCD rounds
  // covering every (channel, slice)
  if (grid <= 0 || grid % (S.SX * kXcds) != 0 || static_cast<int64_t>(grid / S.SX) < static_cast<int64_t>(a.n_chan) * a.slices)
    return hipErrorInvalidValue;
  const size_t lds = fused_lds_bytes(N, V, a.n_weights, a.n_ant);
  hipError_t err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (err != hipSuccess) return err;
  void* args[] = {const_cast<FusedArgs*>(&a)};
  return hipLaunchKernel(k, dim3(grid), dim3(S.NT), args, lds, st);
}

namespace {

template <int N, int V, bool CI4, int WPS>
const void* adjoint_fused_symbol() {
  return reinterpret_cast<const void*>(adjoint_fused_kernel<N, V, CI4, WPS>);
}

template <int N, int V, int WPS>
const void* adjoint_fused_symbol_w(bool ci4) {
  return ci4 ? adjoint_fused_symbol<N, V, true, WPS>() : adjoint_fused_symbol<N, V, false, WPS>();
}

template <int N, int V>
const void* adjoint_fused_symbol_v(bool ci4, int wps) {
  if constexpr (frame_shape(N, V).N == N) {
    if (wps == 1) return adjoint_fused_symbol_w<N, V, 1>(ci4);
    if constexpr (N == 128 || N == 256)
      if (wps == 2) return adjoint_fused_symbol_w<N, V, 2>(ci4);
    if constexpr (N == 128)
      if (wps == 3) return adjoint_fused_symbol_w<N, V, 3>(ci4);
  }
  return nullptr;
}

const void* adjoint_fused_kernel_symbol(int N, int V, bool ci4, int wps) {
  auto pick = [&](auto nc) -> const void* {
    constexpr int NN = decltype(nc)::value;
    return V == 0 ? adjoint_fused_symbol_v<NN, 0>(ci4, wps) : V == 1 ? adjoint_fused_symbol_v<NN, 1>(ci4, wps) : nullptr;
  };
  switch (N) {
    case 8: return pick(std::integral_constant<int, 8>{});
    case 16: return pick(std::integral_constant<int, 16>{});
    case 32: return pick(std::integral_constant<int, 32>{});
    case 64: return pick(std::integral_constant<int, 64>{});
    case 128: return pick(std::integral_constant<int, 128>{});
    case 256: return pick(std::integral_constant<int, 256>{});
    default: return nullptr;
  }
}

}  // namespace

int adjoint_waves_max(int N) { return N == 128 ? 3 : N == 256 ? 2 : 1; }

size_t fused_lane_values(int N, int V) {
  auto go = [&](auto nc, auto vc) -> size_t {
    constexpr int NN = decltype(nc)::value, VV = decltype(vc)::value;
    if constexpr (frame_shape(NN, VV).N == NN) {
      using C = FT<NN, VV>;
      return static_cast<size_t>(C::SX) * C::NACC * C::NT;
    } else {
      return 0;
    }
  };
  auto pick = [&](auto nc) -> size_t {
    return V == 0 ? go(nc, std::integral_constant<int, 0>{}) : V == 1 ? go(nc, std::integral_constant<int, 1>{}) : 0;
  };
  switch (N) {
    case 8: return pick(std::integral_constant<int, 8>{});
    case 16: return pick(std::integral_constant<int, 16>{});
    case 32: return pick(std::integral_constant<int, 32>{});
    case 64: return pick(std::integral_constant<int, 64>{});
    case 128: return pick(std::integral_constant<int, 128>{});
    case 256: return pick(std::integral_constant<int, 256>{});
    default: return 0;
  }
}

hipError_t launch_adjoint_sensitivity(const float* R, int N, int V, int n_chan, float* Rl, hipStream_t st) {
  auto go = [&](auto nc, auto vc) -> hipError_t {
    constexpr int NN = decltype(nc)::value, VV = decltype(vc)::value;
    if constexpr (frame_shape(NN, VV).N == NN) {
      using C = FT<NN, VV>;
      const size_t n = static_cast<size_t>(C::SX) * C::NACC * C::NT * n_chan;
      hipLaunchKernelGGL((adjoint_sensitivity_kernel<NN, VV>), dim3(blocks_for(n)), dim3(256), 0, st, R, n_chan, Rl);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  };
  auto pick = [&](auto nc) -> hipError_t {
    return V == 0 ? go(nc, std::integral_constant<int, 0>{}) : V == 1 ? go(nc, std::integral_constant<int, 1>{})
                                                                      : hipErrorInvalidValue;
  };
  switch (N) {
    case 8: return pick(std::integral_constant<int, 8>{});
    case 16: return pick(std::integral_constant<int, 16>{});
    case 32: return pick(std::integral_constant<int, 32>{});
    case 64: return pick(std::integral_constant<int, 64>{});
    case 128: return pick(std::integral_constant<int, 128>{});
    case 256: return pick(std::integral_constant<int, 256>{});
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_fused(const AdjFusedArgs& a, int N, int V, bool ci4, int wps, int grid, hipStream_t st) {
  const void* k = adjoint_fused_kernel_symbol(N, V, ci4, wps);
  if (!k) return hipErrorInvalidValue;
  const FrameShape S = frame_shape(N, V);
  const size_t lds = fused_lds_bytes(N, V, a.n_weights, a.n_ant);
  hipError_t err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (err != hipSuccess) return err;
  void* args[] = {const_cast<AdjFusedArgs*>(&a)};
  return hipLaunchKernel(k, dim3(grid), dim3(S.NT), args, lds, st);
}

int adjoint_fused_blocks_per_cu(int N, int V, bool ci4, int wps, size_t lds) {
  const void* k = adjoint_fused_kernel_symbol(N, V, ci4, wps);
  if (!k) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, frame_shape(N, V).NT, lds) != hipSuccess) return 1;
  return n;
}

hipError_t launch_antenna_power(const void* E, bool ci4, int64_t n_time, int n_chan, int n_ant, double* Q,
                                hipStream_t st) {
  const dim3 grid((n_ant + 255) / 256, n_chan);
  if (ci4) hipLaunchKernelGGL(antenna_power_kernel<true>, grid, dim3(256), 0, st, E, n_time, n_chan, n_ant, Q);
  else hipLaunchKernelGGL(antenna_power_kernel<false>, grid, dim3(256), 0, st, E, n_time, n_chan, n_ant, Q);
  return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const double2* Dp, int parts, int n_chan, int n_ant, double2* D, hipStream_t st) {
  const size_t n = static_cast<size_t>(n_chan) * n_ant;
  hipLaunchKernelGGL(adjoint_reduce_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, Dp, parts,
                     n, D);
  return hipGetLastError();
}

int fused_blocks_per_cu(int N, int V, bool ci4, size_t lds) {
  // (both antenna variants are sized for the same waves per SIMD)
  const void* k = fused_kernel_symbol(N, V, ci4, false);
  if (!k) return 0;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, frame_shape(N, V).NT, lds) != hipSuccess) return 0;
  return blocks;
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(static_cast<size_t>(a.N) * a.N * a.n_chan / 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_grid(const GridArgs& a, bool ci4, hipStream_t st) {
  const size_t lds = sizeof(float2) * (a.n_ant + a.n_taps);
  const unsigned frames = static_cast<unsigned>(a.n_time * a.n_chan);  // checked < 2^31 by the caller
  if (ci4)
    hipLaunchKernelGGL(grid_kernel<true>, dim3(frames), dim3(256), lds, st, a);
  else
    hipLaunchKernelGGL(grid_kernel<false>, dim3(frames), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_self_power(const GridArgs& a, bool ci4, hipStream_t st) {
  if (ci4)
    hipLaunchKernelGGL(self_power_kernel<true>, dim3(a.n_chan), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(self_power_kernel<false>, dim3(a.n_chan), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fft2(const Fft2Args& a, int N, int64_t n_frames, hipStream_t st) {
  switch (N) {
    case 8: return launch_fft2_t<8>(a, n_frames, st);
    case 16: return launch_fft2_t<16>(a, n_frames, st);
    case 32: return launch_fft2_t<32>(a, n_frames, st);
    case 64: return launch_fft2_t<64>(a, n_frames, st);
    case 128: return launch_fft2_t<128>(a, n_frames, st);
    case 256: return launch_fft2_t<256>(a, n_frames, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_detect(const DetectArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(detect_kernel, dim3(blocks_for(static_cast<size_t>(a.N) * a.N * a.n_chan)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(static_cast<size_t>(a.N) * a.N * a.n_chan)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  const unsigned blocks = static_cast<unsigned>(std::min<size_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(zero_kernel, dim3(blocks ? blocks : 1), dim3(256), 0, st, static_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

hipError_t launch_adjoint_fft2(const AdjFftArgs& a, int N, int64_t n_frames, hipStream_t st) {
  auto go = [&](auto nc) -> hipError_t {
    constexpr int NN = decltype(nc)::value;
    using C = FT<NN, 0>;
    const size_t lds = sizeof(float2) * (static_cast<size_t>(C::GRID) + C::TWR + C::TWC);
    auto k = adjoint_fft2_kernel<NN>;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(n_frames * C::SX)), dim3(C::NT), lds, st, a);
    return hipGetLastError();
  };
  switch (N) {
    case 8: return go(std::integral_constant<int, 8>{});
    case 16: return go(std::integral_constant<int, 16>{});
    case 32: return go(std::integral_constant<int, 32>{});
    case 64: return go(std::integral_constant<int, 64>{});
    case 128: return go(std::integral_constant<int, 128>{});
    case 256: return go(std::integral_constant<int, 256>{});
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_degrid(const DegridArgs& a, bool ci4, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((a.n_ant + 255) / 256), static_cast<unsigned>(a.n_chan));
  if (ci4)
    hipLaunchKernelGGL(degrid_kernel<true>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(degrid_kernel<false>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_grad_final(const GradFinalArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(grad_final_kernel, dim3(a.n_chan), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace moff
