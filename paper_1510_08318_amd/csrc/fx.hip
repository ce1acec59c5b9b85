// Visibility-route (FX) imaging of one integration on the device, for
// cross-checks of the MOFF image by the paper's other method (Sec. 2: the
// time-averaged cross-products of the calibrated antenna fields, eq. cc-vis,
// gridded with each pair's power response, the cross-correlation of the two
// aperture illuminations, eq. e-field-conv, and transformed once, eq.
// dirty-image-FX, give the MOFF image; with the zero-spacing a == b terms left
// out it equals the image with the antennas' self power removed).
//
//   fx_correlate_kernel  V[c][a][b] = sum_t e_a conj(e_b), e = g E, for a <= b
//                        (the upper triangle; V is Hermitian): float32
//                        matrix-core products over 32-sample chunks, chunks
//                        summed in float64 (complex64 samples);
//                        fx_correlate_i8_kernel: exact integer products on the
//                        matrix cores (4+4-bit samples)
//   fx_bin_kernel        H[c][pq][dy][dx] = sum of V[c][a][b] over the pairs of
//                        table types (p, q) whose footprints are offset by
//                        (dy, dx) - (L - 1) cells (plan-time CSR, fixed order);
//                        half the cells are summed, their mirrors
//                        H[qp][-dy][-dx] written as the conjugates
//   fx_lag_kernel        R[c][ly][lx] = sum_pq sum_(u,v) X_pq[u][v]
//                        H[c][pq][ly - u + k_q - 1][lx - v + k_q - 1]  (LDS-tiled;
//                        half the cells, their mirrors written as conjugates)
//   fx_row_kernel        Z[c][ly][q] = sum_lx R[c][ly][lx] w^((lx - L + 1)(q - N/2))
//                        (rows up to the zero lag; the others are conjugates)
//   fx_col_kernel        I[c][r][q] = scale Re sum_ly w^((ly - L + 1)(r - N/2)) Z[c][ly][q]
//                        (real, two columns per complex transform)
//                        (both as N-point radix-2 transforms in LDS, float32)
//
// w = exp(+2 pi i / N); lags span -(L - 1) .. L - 1, so the image comes out in
// the same pixel order as the MOFF image.  Every sum runs in a fixed order
// (no atomics); the correlator and the binning accumulate in float64, each
// pair response's lag sum in float32 (the pairs in float64), and the two
// transform passes run in float32; intermediate arrays are float32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "fx.h"
#include "fx_tables.h"
#include "ingest.h"

namespace moff {

namespace {

constexpr int kFxChunk = 32;   // time samples staged per step
constexpr unsigned kFxXcds = 8;  // accelerator dies (XCDs), each with its own L2

// Workgroups go to the XCDs round-robin by linear index.  For a 1-D grid of
// kFxXcds * ceil(n / kFxXcds) * per blocks over n channels of `per` blocks
// each, the channel of block b and its index within the channel: all blocks of
// a channel share one residue mod kFxXcds, so one XCD's L2 serves the data of
// that channel.  Returns false for the padding blocks.
__device__ __forceinline__ bool xcd_channel(unsigned b, unsigned per, int n, int* ch, unsigned* j) {
  const unsigned xcd = b % kFxXcds, s = b / kFxXcds;
  *ch = static_cast<int>(xcd + kFxXcds * (s / per));
  *j = s % per;
  return *ch < n;
}
inline size_t xcd_grid(size_t per, int n) { return per * kFxXcds * ((static_cast<size_t>(n) + kFxXcds - 1) / kFxXcds); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace

// Complex64 samples, on the matrix cores in float32 (v_mfma_f32_16x16x4_f32).
// The visibility matrix is Hermitian, V_ba = conj(V_ab), and the binning reads
// its upper triangle only, so only the tiles on and above the diagonal are
// formed.  One workgroup per (64 x 64 antenna tile, channel), four waves
// of a 32 x 32 sub-tile each (2 x 2 blocks of 16 x 16).  The complex product
// is two real contractions over k = (sample, part):
//   Re V_ab = sum_k A_ak B_bk,   A = (re e, im e) of antenna a, B the same of b,
//   Im V_ab = sum_k A'_ak B_bk,  A' = (im e, -re e) of antenna a.
// Lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] with the same k = l / 16
// (sample 2 step + k / 2, part k % 2), so each (sample, part) is summed once
// whatever order the instruction takes its contraction index in; the
// accumulators hold D[4 (l / 16) + v][l % 16].  Each 32-sample chunk is summed
// in float32 and the chunks in float64.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kC64Tile = 64;               // antennas per side of a tile
constexpr int kC64Pitch = kC64Tile + 16;   // float2 per LDS row: two samples' 16 rows hit distinct banks

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void fx_correlate_kernel(FxArgs a) {
  __shared__ float2 ea[kFxChunk][kC64Pitch], eb[kFxChunk][kC64Pitch];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave >> 1, wb = wave & 1, r16 = lane & 15, kk = lane >> 4;
  const int na = a.n_ant, n_tiles = (na + kC64Tile - 1) / kC64Tile;
  int cl;
  unsigned tri;
  if (!xcd_channel(blockIdx.x, static_cast<unsigned>(n_tiles * (n_tiles + 1) / 2), a.n_launch, &cl, &tri)) return;
  int t = static_cast<int>(tri), ta = 0;      // upper-triangle tile (ta, tb), tb >= ta
  while (ta < n_tiles && t >= n_tiles - ta) {
    t -= n_tiles - ta;
    ++ta;
  }
  if (ta >= n_tiles) return;                  // beyond the triangle (the launch has none)
  const int tb = ta + t;
  const int a0 = ta * kC64Tile, b0 = tb * kC64Tile, c = a.c0 + cl;
  const float2* E = reinterpret_cast<const float2*>(a.E);
  double acc[2][2][4][2] = {};
  // staging: thread = (antenna an, samples sg + kC64Rows i), so each thread
  // keeps its two antennas' gains for the whole integration
  constexpr int kC64Rows = 256 / kC64Tile, kC64Per = kFxChunk / kC64Rows;
  const int an = tid % kC64Tile, sg = tid / kC64Tile;
  const int ia = a0 + an, ib = b0 + an;
  const float2 one = make_float2(1.f, 0.f);
  const float2 ga = (a.gains && ia < na) ? a.gains[static_cast<size_t>(c) * na + ia] : one;
  const float2 gb = (a.gains && ib < na) ? a.gains[static_cast<size_t>(c) * na + ib] : one;
  float2 pa[kC64Per], pb[kC64Per];
  auto load_chunk = [&](int64_t t0) {   // all of a chunk's loads in flight at once
#pragma unroll
    for (int i = 0; i < kC64Per; ++i) {
      const int64_t ts = t0 + sg + kC64Rows * i;
      const size_t base = (static_cast<size_t>(ts) * a.n_chan + c) * na;
      // out-of-range samples load element 0 (always valid) and read as zero
      const bool oka = ts < a.n_time && ia < na, okb = ts < a.n_time && ib < na;
      const float2 va = E[oka ? base + ia : size_t(0)], vb = E[okb ? base + ib : size_t(0)];
      pa[i] = oka ? va : make_float2(0.f, 0.f);
      pb[i] = okb ? vb : make_float2(0.f, 0.f);
    }
  };
  for (int64_t t0 = 0; t0 < a.n_time; t0 += kFxChunk) {
    load_chunk(t0);
#pragma unroll
    for (int i = 0; i < kC64Per; ++i) {
      ea[sg + kC64Rows * i][an] = cmul(ga, pa[i]);
      eb[sg + kC64Rows * i][an] = cmul(gb, pb[i]);
    }
    __syncthreads();
    f32x4 re[2][2], im[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        re[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        im[i][j] = re[i][j];
      }
    const bool imag_part = kk & 1;
#pragma unroll 4
    for (int step = 0; step < kFxChunk / 2; ++step) {
      const int sm = 2 * step + (kk >> 1);
      float A[2], Ap[2], B[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float2 x = ea[sm][32 * wa + 16 * i + r16];
        A[i] = imag_part ? x.y : x.x;
        Ap[i] = imag_part ? -x.x : x.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float2 y = eb[sm][32 * wb + 16 * j + r16];
        B[j] = imag_part ? y.y : y.x;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[i], B[j], re[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ap[i], B[j], im[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[i][j][v][0] += re[i][j][v];
          acc[i][j][v][1] += im[i][j][v];
        }
    __syncthreads();
  }
  float2* V = a.V + static_cast<size_t>(cl) * na * na;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ia = a0 + 32 * wa + 16 * i + 4 * kk + v, ib = b0 + 32 * wb + 16 * j + r16;
        if (ia >= na || ib >= na) continue;
        const float x = static_cast<float>(acc[i][j][v][0]), y = static_cast<float>(acc[i][j][v][1]);
        V[static_cast<size_t>(ia) * na + ib] = make_float2(x, y);
      }
}

// 4+4-bit samples: the cross-products are exact integer sums, formed on the
// matrix cores (v_mfma_i32_16x16x64_i8, int32 accumulation) from the raw
// samples; the gains are constant over the integration and are applied once,
// V_ab = g_a conj(g_b) sum_t E_a conj(E_b), in float64.  One workgroup per
// (64 x 64 antenna tile on or above the diagonal, channel), four waves of a
// 32 x 32 sub-tile each (2 x 2 blocks of 16 x 16).  Per 64-sample step the
// real and imaginary parts of both antenna blocks are staged in LDS as int8
// rows [antenna][sample], and each wave runs four products (re.re, im.im,
// im.re, re.im) per block; the next step's samples are loaded into registers
// while the current step's products run.  A and B take their samples in the
// same lane order, so the sum covers each sample once whatever order the
// instruction gives its contraction index; the accumulators hold
// D[4 (l / 16) + j][l % 16].
typedef int i32x4 __attribute__((ext_vector_type(4)));
constexpr int kI8Step = 64;                 // samples per step
constexpr int kI8Pitch = kI8Step + 16;      // LDS row bytes: 16-byte operand reads of 16 rows hit distinct banks

constexpr int kI8Blocks = 2;                          // 16 x 16 blocks per wave and side
constexpr int kI8Tile = 32 * kI8Blocks;               // antennas per side of a tile
constexpr int kI8PerThread = kI8Step * kI8Tile / 256;   // samples per thread and step, per block

__global__ __launch_bounds__(256) void fx_correlate_i8_kernel(FxArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t pl[4][kI8Tile][kI8Pitch];   // re A, im A, re B, im B
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int na = a.n_ant, n_tiles = (na + kI8Tile - 1) / kI8Tile;
  int cl;
  unsigned tri;
  if (!xcd_channel(blockIdx.x, static_cast<unsigned>(n_tiles * (n_tiles + 1) / 2), a.n_launch, &cl, &tri)) return;
  int t = static_cast<int>(tri), ta = 0;      // upper-triangle tile (ta, tb), tb >= ta
  while (ta < n_tiles && t >= n_tiles - ta) {
    t -= n_tiles - ta;
    ++ta;
  }
  if (ta >= n_tiles) return;                  // beyond the triangle (the launch has none)
  const int a0 = ta * kI8Tile, b0 = (ta + t) * kI8Tile, c = a.c0 + cl;
  const int8_t* E = reinterpret_cast<const int8_t*>(a.E);
  const size_t tstride = static_cast<size_t>(a.n_chan) * na;
  // staging: thread = (antenna an, group tg of kI8PerThread samples) for both blocks
  const int an = tid % kI8Tile, tg = tid / kI8Tile;   // tg < 256 / kI8Tile
  // this wave's sub-tile and its operand rows
  const int ah = w >> 1, bh = w & 1, l16 = lane & 15, g = lane >> 4;
  i32x4 acc[kI8Blocks][kI8Blocks][4];
#pragma unroll
  for (int i = 0; i < kI8Blocks; ++i)
#pragma unroll
    for (int j = 0; j < kI8Blocks; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[i][j][q] = i32x4{0, 0, 0, 0};
  int8_t nxt[2][kI8PerThread];
  auto load_step = [&](int64_t t0) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int ant = (blk ? b0 : a0) + an;
#pragma unroll
      for (int i = 0; i < kI8PerThread; ++i) {
        // out-of-range samples load element 0 (always valid) and read as zero:
        // no branch around each load
        const int64_t ts = t0 + kI8PerThread * tg + i;
        const bool ok = ant < na && ts < a.n_time;
        const int8_t v = E[ok ? static_cast<size_t>(ts) * tstride + static_cast<size_t>(c) * na + ant : size_t(0)];
        nxt[blk][i] = ok ? v : int8_t(0);
      }
    }
  };
  load_step(0);
  for (int64_t t0 = 0; t0 < a.n_time; t0 += kI8Step) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      uint64_t xr[kI8Blocks] = {}, xi[kI8Blocks] = {};
#pragma unroll
      for (int i = 0; i < kI8PerThread; ++i) {
        const int8_t byte = nxt[blk][i];
        const int8_t re = static_cast<int8_t>(byte >> 4);
        const int8_t im = static_cast<int8_t>(static_cast<int8_t>(byte << 4) >> 4);
        xr[i / 8] |= static_cast<uint64_t>(static_cast<uint8_t>(re)) << (8 * (i % 8));
        xi[i / 8] |= static_cast<uint64_t>(static_cast<uint8_t>(im)) << (8 * (i % 8));
      }
      uint64_t* dr = reinterpret_cast<uint64_t*>(&pl[2 * blk][an][kI8PerThread * tg]);
      uint64_t* di = reinterpret_cast<uint64_t*>(&pl[2 * blk + 1][an][kI8PerThread * tg]);
#pragma unroll
      for (int h = 0; h < kI8Blocks; ++h) {
        dr[h] = xr[h];
        di[h] = xi[h];
      }
    }
    __syncthreads();
    if (t0 + kI8Step < a.n_time) load_step(t0 + kI8Step);   // in flight during the products
    i32x4 ar[kI8Blocks], ai[kI8Blocks], br[kI8Blocks], bi[kI8Blocks];
#pragma unroll
    for (int i = 0; i < kI8Blocks; ++i) {
      ar[i] = *reinterpret_cast<const i32x4*>(&pl[0][16 * kI8Blocks * ah + 16 * i + l16][16 * g]);
      ai[i] = *reinterpret_cast<const i32x4*>(&pl[1][16 * kI8Blocks * ah + 16 * i + l16][16 * g]);
      br[i] = *reinterpret_cast<const i32x4*>(&pl[2][16 * kI8Blocks * bh + 16 * i + l16][16 * g]);
      bi[i] = *reinterpret_cast<const i32x4*>(&pl[3][16 * kI8Blocks * bh + 16 * i + l16][16 * g]);
    }
#pragma unroll
    for (int i = 0; i < kI8Blocks; ++i)
#pragma unroll
      for (int j = 0; j < kI8Blocks; ++j) {
        acc[i][j][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ar[i], br[j], acc[i][j][0], 0, 0, 0);
        acc[i][j][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai[i], bi[j], acc[i][j][1], 0, 0, 0);
        acc[i][j][2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai[i], br[j], acc[i][j][2], 0, 0, 0);
        acc[i][j][3] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ar[i], bi[j], acc[i][j][3], 0, 0, 0);
      }
    __syncthreads();
  }
  float2* V = a.V + static_cast<size_t>(cl) * na * na;
#pragma unroll
  for (int i = 0; i < kI8Blocks; ++i)
#pragma unroll
    for (int j = 0; j < kI8Blocks; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ia = a0 + 16 * kI8Blocks * ah + 16 * i + 4 * g + e, ib = b0 + 16 * kI8Blocks * bh + 16 * j + l16;
        if (ia >= na || ib >= na) continue;
        // E_a conj(E_b) = (xa xb + ya yb) + i (ya xb - xa yb)
        const double vr = static_cast<double>(acc[i][j][0][e]) + acc[i][j][1][e];
        const double vi = static_cast<double>(acc[i][j][2][e]) - acc[i][j][3][e];
        double zr = vr, zi = vi;
        if (a.gains) {
          const float2 ga = a.gains[static_cast<size_t>(c) * na + ia], gb = a.gains[static_cast<size_t>(c) * na + ib];
          // g_a conj(g_b)
          const double gr = static_cast<double>(ga.x) * gb.x + static_cast<double>(ga.y) * gb.y;
          const double gi = static_cast<double>(ga.y) * gb.x - static_cast<double>(ga.x) * gb.y;
          zr = gr * vr - gi * vi;
          zi = gr * vi + gi * vr;
        }
        V[static_cast<size_t>(ia) * na + ib] = make_float2(static_cast<float>(zr), static_cast<float>(zi));
      }
}

constexpr int kFxBinBatch = 8;   // pair loads in flight per thread of the binning

// One thread per (channel, type pair, offset cell).  The thread of a cell at
// or before its mirror (types swapped, offset negated) sums the cell's pairs
// and writes the mirror cell as the conjugate; the thread of a later cell has
// nothing to do.
__global__ __launch_bounds__(256) void fx_bin_kernel(FxArgs a) {
  const int nl2 = a.NL * a.NL;
  const size_t cells = static_cast<size_t>(a.n_types) * a.n_types * nl2;
  int c;
  unsigned blk;
  if (!xcd_channel(blockIdx.x, static_cast<unsigned>((cells + 255) / 256), a.n_launch, &c, &blk)) return;
  const size_t i = static_cast<size_t>(blk) * 256 + threadIdx.x;
  if (i >= cells) return;
  const int tp = static_cast<int>(i / nl2), off = static_cast<int>(i % nl2);
  const size_t m = static_cast<size_t>((tp % a.n_types) * a.n_types + tp / a.n_types) * nl2 + (nl2 - 1 - off);
  if (m < i) return;
  const float2* V = a.V + static_cast<size_t>(c) * a.n_ant * a.n_ant;
  double x = 0.0, y = 0.0;
  // Rows of short, redundant baselines hold hundreds of pairs: loads go out
  // kFxBinBatch at a time (indices, then visibilities) and are summed in the
  // same order as one at a time.
  int k = a.pair_ptr[i];
  const int k1 = a.pair_ptr[i + 1];
  for (; k + kFxBinBatch <= k1; k += kFxBinBatch) {
    uint32_t e[kFxBinBatch];
    float2 v[kFxBinBatch];
#pragma unroll
    for (int j = 0; j < kFxBinBatch; ++j) e[j] = static_cast<uint32_t>(a.pair_ab[k + j]);
#pragma unroll
    for (int j = 0; j < kFxBinBatch; ++j) v[j] = V[e[j] & ~kFxConjBit];
#pragma unroll
    for (int j = 0; j < kFxBinBatch; ++j) {
      x += v[j].x;
      y += (e[j] & kFxConjBit) ? -v[j].y : v[j].y;
    }
  }
  for (; k < k1; ++k) {
    const uint32_t e = static_cast<uint32_t>(a.pair_ab[k]);
    const float2 v = V[e & ~kFxConjBit];
    x += v.x;
    y += (e & kFxConjBit) ? -v.y : v.y;
  }
  float2* H = a.H + static_cast<size_t>(c) * cells;
  H[i] = make_float2(static_cast<float>(x), static_cast<float>(y));
  if (m != i) H[m] = make_float2(static_cast<float>(x), static_cast<float>(-y));
}

// One workgroup per (16 x 64 block of lag cells, channel); each thread owns
// four horizontally adjacent cells.  Per type pair the block's window of H
// (with a halo of the pair response's side) and the response itself are
// staged in LDS; cells of H outside the lag grid read as zero.  Along a
// response row the four cells' window values slide by one column per tap, so
// a row of `side` taps reads side + 3 window values instead of 4 side.  The
// pair responses obey X_qp(-u) = conj X_pq(u) and the binned sums
// H_qp(-d) = conj H_pq(d) (centred offsets), so the lag grid obeys
// R(-l) = conj R(l): blocks past the zero lag return at once, and each cell
// before it also writes its mirror.
constexpr int kLagRows = 16, kLagCols = 64, kLagCells = 4;   // block of lag cells; cells per thread

__global__ __launch_bounds__(256) void fx_lag_kernel(FxArgs a) {
  extern __shared__ float2 fx_lds[];
  const int NL = a.NL, nt = a.n_types, c = blockIdx.z;
  const int hw = kLagCols + a.xs - 1;             // window row pitch (widest window)
  float2* Ht = fx_lds;                            // [kLagRows + xs - 1][hw]
  float2* Xt = fx_lds + (kLagRows + a.xs - 1) * hw;   // [side][side]
  const int tyl = threadIdx.x / (kLagCols / kLagCells), txg = threadIdx.x % (kLagCols / kLagCells);
  const int ty0 = blockIdx.y * kLagRows, tx0 = blockIdx.x * kLagCols;
  const int mid = NL / 2;                         // the zero lag, L - 1
  if (ty0 > mid || (ty0 == mid && tx0 > mid)) return;   // no cell at or before its mirror
  const size_t plane = static_cast<size_t>(NL) * NL;
  double x[kLagCells] = {}, y[kLagCells] = {};
  for (int tp = 0; tp < nt * nt; ++tp) {
    const int kb = a.ktype_k[tp % nt], side = a.ktype_k[tp / nt] + kb - 1;
    const int ey = kLagRows + side - 1, ex = kLagCols + side - 1;
    const int hy0 = ty0 + kb - side, hx0 = tx0 + kb - side;
    const float2* H = a.H + (static_cast<size_t>(c) * nt * nt + tp) * plane;
    const float2* X = a.xcorr + static_cast<size_t>(tp) * a.xs * a.xs;
    __syncthreads();   // the previous pair's windows are no longer read
    for (int i = threadIdx.x; i < ey * ex; i += blockDim.x) {
      const int hy = hy0 + i / ex, hx = hx0 + i % ex;
      Ht[(i / ex) * hw + i % ex] =
          (hy >= 0 && hy < NL && hx >= 0 && hx < NL) ? H[static_cast<size_t>(hy) * NL + hx] : make_float2(0.f, 0.f);
    }
    for (int i = threadIdx.x; i < side * side; i += blockDim.x) Xt[i] = X[(i / side) * a.xs + i % side];
    __syncthreads();
    // cell (tyl, 4 txg + j) at response tap (u, v) reads window cell
    // (tyl - u + side - 1, 4 txg + j - v + side - 1); one pair's response sum
    // in float32, the pairs combined in float64
    float px[kLagCells] = {}, py[kLagCells] = {};
    for (int u = 0; u < side; ++u) {
      const float2* hrow = Ht + (tyl - u + side - 1) * hw + kLagCells * txg + side - 1;
      float2 h0 = hrow[0], h1 = hrow[1], h2 = hrow[2], h3 = hrow[3];
      for (int v = 0; v < side; ++v) {
        const float2 w = Xt[u * side + v];
        px[0] = fmaf(w.x, h0.x, fmaf(-w.y, h0.y, px[0]));
        py[0] = fmaf(w.x, h0.y, fmaf(w.y, h0.x, py[0]));
        px[1] = fmaf(w.x, h1.x, fmaf(-w.y, h1.y, px[1]));
        py[1] = fmaf(w.x, h1.y, fmaf(w.y, h1.x, py[1]));
        px[2] = fmaf(w.x, h2.x, fmaf(-w.y, h2.y, px[2]));
        py[2] = fmaf(w.x, h2.y, fmaf(w.y, h2.x, py[2]));
        px[3] = fmaf(w.x, h3.x, fmaf(-w.y, h3.y, px[3]));
        py[3] = fmaf(w.x, h3.y, fmaf(w.y, h3.x, py[3]));
        h3 = h2;
        h2 = h1;
        h1 = h0;
        if (v + 1 < side) h0 = hrow[-(v + 1)];
      }
    }
#pragma unroll
    for (int j = 0; j < kLagCells; ++j) {
      x[j] += px[j];
      y[j] += py[j];
    }
  }
  const int ly = ty0 + tyl;
  float2* R = a.R + static_cast<size_t>(c) * plane;
#pragma unroll
  for (int j = 0; j < kLagCells; ++j) {
    const int lx = tx0 + kLagCells * txg + j;
    const bool canonical = ly < mid || (ly == mid && lx <= mid);
    if (ly >= NL || lx >= NL || !canonical) continue;
    R[static_cast<size_t>(ly) * NL + lx] = make_float2(static_cast<float>(x[j]), static_cast<float>(y[j]));
    if (ly != mid || lx != mid)
      R[static_cast<size_t>(NL - 1 - ly) * NL + (NL - 1 - lx)] =
          make_float2(static_cast<float>(x[j]), static_cast<float>(-y[j]));
  }
}

// Radix-2 decimation-in-time transform, in place, of `lines` interleaved lines
// of N points in LDS (point n of line k at X[n * lines + k]) loaded in
// bit-reversed order: X[m] = sum_n x[n] w^(n m), w = tw[1] = exp(+2 pi i / N).
__device__ __forceinline__ void fft_lines(float2* X, const float2* tw, int N, int lines) {
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len >> 1, step = N / len;
    for (int b = threadIdx.x; b < lines * (N >> 1); b += blockDim.x) {
      const int k = b % lines, j = b / lines;
      const int i0 = (j / half) * len + (j % half), i1 = i0 + half;
      const float2 u = X[i0 * lines + k], v = cmul(X[i1 * lines + k], tw[(j % half) * step]);
      X[i0 * lines + k] = make_float2(u.x + v.x, u.y + v.y);
      X[i1 * lines + k] = make_float2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bit_reverse(int n, int bits) { return static_cast<int>(__brev(static_cast<unsigned>(n)) >> (32 - bits)); }

// Lag d = j - (L - 1) of a lag-grid line goes to point n = d mod N with the
// factor (-1)^d, so that the transform's output index is the pixel index:
// w^(d (q - N/2)) = (-1)^d w^(d q).  Point N/2 (d = -L) stays zero.
__device__ __forceinline__ float2 lag_point(const float2* line, int n, int N, int L) {
  const int d = n < N / 2 ? n : n - N;
  if (d < -(L - 1) || d > L - 1) return make_float2(0.f, 0.f);
  const float2 v = line[d + L - 1];
  return (d & 1) ? make_float2(-v.x, -v.y) : v;
}

constexpr int kFxRowLines = 8;   // lag rows per workgroup of the row pass

// Row pass: one workgroup per (block of kFxRowLines lag rows, channel).  With
// R(-l) = conj R(l), the transform of lag row NL - 1 - ly is the conjugate of
// that of row ly (same pixel column), so only rows up to the zero lag L - 1
// are transformed and each row before it also writes its mirror.
__global__ __launch_bounds__(256) void fx_row_kernel(FxArgs a) {
  extern __shared__ float2 fx_lds[];
  const int N = a.N, NL = a.NL, L = a.L, c = blockIdx.y, ly0 = blockIdx.x * kFxRowLines;
  const int bits = 31 - __clz(N);
  float2* X = fx_lds;                       // [N][kFxRowLines]
  float2* tw = fx_lds + N * kFxRowLines;    // [N]
  for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = a.tw[i];
  const float2* R = a.R + static_cast<size_t>(c) * NL * NL;
  for (int i = threadIdx.x; i < kFxRowLines * N; i += blockDim.x) {
    const int k = i / N, n = i % N, ly = ly0 + k;
    X[bit_reverse(n, bits) * kFxRowLines + k] =
        ly < NL ? lag_point(R + static_cast<size_t>(ly) * NL, n, N, L) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lines(X, tw, N, kFxRowLines);
  float2* Z = a.Z + static_cast<size_t>(c) * NL * N;
  for (int i = threadIdx.x; i < kFxRowLines * N; i += blockDim.x) {
    const int k = i / N, q = i % N, ly = ly0 + k;
    if (ly > L - 1) continue;   // written by its mirror row
    const float2 v = X[q * kFxRowLines + k];
    Z[static_cast<size_t>(ly) * N + q] = v;
    if (ly < L - 1) Z[static_cast<size_t>(NL - 1 - ly) * N + q] = make_float2(v.x, -v.y);
  }
}

// Column pass: one workgroup per (block of 2 cw image columns, channel).  Each
// column of Z is Hermitian in the lag (Z(-l, q) = conj Z(l, q)), so its
// transform is real: columns q and q + cw go through one complex transform as
// Z(., q) + i Z(., q + cw), and the real and imaginary parts of the result are
// the two image columns.  The lag columns are gathered through lag_point's
// mapping, and the scaled results written as row segments of the image.
__device__ __forceinline__ int fx_col_width(int N) { return N < 16 ? 1 : (N / 8 < 16 ? N / 8 : 16); }

__global__ __launch_bounds__(256) void fx_col_kernel(FxArgs a) {
  extern __shared__ float2 fx_lds[];
  const int N = a.N, NL = a.NL, L = a.L, c = blockIdx.y;   // c: channel within the launch
  const int cw = fx_col_width(N), q0 = blockIdx.x * 2 * cw, bits = 31 - __clz(N);
  float2* X = fx_lds;                       // [N][cw]
  float2* tw = fx_lds + N * cw;             // [N]
  for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = a.tw[i];
  const float2* Z = a.Z + static_cast<size_t>(c) * NL * N;
  for (int i = threadIdx.x; i < cw * N; i += blockDim.x) {
    const int n = i / cw, k = i % cw;
    const int d = n < N / 2 ? n : n - N;
    float2 v = make_float2(0.f, 0.f);
    if (d >= -(L - 1) && d <= L - 1) {
      const float2 z1 = Z[static_cast<size_t>(d + L - 1) * N + q0 + k];
      const float2 z2 = Z[static_cast<size_t>(d + L - 1) * N + q0 + cw + k];
      v = make_float2(z1.x - z2.y, z1.y + z2.x);   // z1 + i z2
      if (d & 1) v = make_float2(-v.x, -v.y);
    }
    X[bit_reverse(n, bits) * cw + k] = v;
  }
  __syncthreads();
  fft_lines(X, tw, N, cw);
  float* out = a.out + static_cast<size_t>(a.c0 + c) * N * N;
  for (int i = threadIdx.x; i < 2 * cw * N; i += blockDim.x) {
    const int r = i / (2 * cw), k = i % (2 * cw);
    const float2 y = X[r * cw + k % cw];
    out[static_cast<size_t>(r) * N + q0 + k] = static_cast<float>((k < cw ? y.x : y.y) * a.scale);
  }
}

hipError_t launch_fx(const FxArgs& a, bool ci4, hipStream_t st) {
  if (a.n_ant < 1 || a.n_launch < 1 || a.n_launch > 65535 || a.c0 < 0 || a.c0 + a.n_launch > a.n_chan || a.N < 8 ||
      a.N > 256 || a.NL != 2 * a.L - 1 || a.n_types < 1 || a.n_types > kMaxTypesDev)
    return hipErrorInvalidValue;
  if (ci4) {
    const size_t nt = static_cast<size_t>((a.n_ant + kI8Tile - 1) / kI8Tile);
    const size_t blocks = xcd_grid(nt * (nt + 1) / 2, a.n_launch);
    if (blocks > 0x7FFFFFFFu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fx_correlate_i8_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a);
  } else {
    const size_t nt = static_cast<size_t>((a.n_ant + kC64Tile - 1) / kC64Tile);
    const size_t blocks = xcd_grid(nt * (nt + 1) / 2, a.n_launch);
    if (blocks > 0x7FFFFFFFu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fx_correlate_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t cells = static_cast<size_t>(a.n_types) * a.n_types * a.NL * a.NL;
  const size_t bin_blocks = xcd_grid((cells + 255) / 256, a.n_launch);
  if (bin_blocks > 0x7FFFFFFFu) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fx_bin_kernel, dim3(static_cast<unsigned>(bin_blocks)), dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned lag_bx = static_cast<unsigned>((a.NL + kLagCols - 1) / kLagCols);
  const unsigned lag_by = static_cast<unsigned>((a.NL + kLagRows - 1) / kLagRows);
  const size_t lag_lds =
      sizeof(float2) * static_cast<size_t>((kLagRows + a.xs - 1) * (kLagCols + a.xs - 1) + a.xs * a.xs);
  hipLaunchKernelGGL(fx_lag_kernel, dim3(lag_bx, lag_by, a.n_launch), dim3(kLagRows * kLagCols / kLagCells), lag_lds,
                     st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t row_lds = sizeof(float2) * static_cast<size_t>(a.N) * (kFxRowLines + 1);
  const unsigned row_blocks = static_cast<unsigned>((a.L + kFxRowLines - 1) / kFxRowLines);   // rows 0 .. L - 1
  hipLaunchKernelGGL(fx_row_kernel, dim3(row_blocks, a.n_launch), dim3(256), row_lds, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int cw = a.N < 16 ? 1 : std::min(a.N / 8, 16);   // fx_col_width
  const size_t col_lds = sizeof(float2) * static_cast<size_t>(a.N) * (cw + 1);
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fx_col_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(col_lds))) != hipSuccess)
    return e;
  hipLaunchKernelGGL(fx_col_kernel, dim3(a.N / (2 * cw), a.n_launch), dim3(256), col_lds, st, a);
  return hipGetLastError();
}

}  // namespace moff
