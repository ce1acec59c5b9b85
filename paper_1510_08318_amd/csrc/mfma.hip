// Reduced-precision MOFF frame transform on the gfx950 matrix cores.
//
// For grids of 64 and 128 the padded 2-D DFT of Sec. 3 is computed as two
// dense complex matrix products (Sec. 6.1 counts the transform as the dominant
// cost; at these sizes the contraction is small enough to run as plain matrix
// products), over the L = N/2 nonzero rows and columns of the zero-padded grid:
//
//   row stage     Z[iy][q] = sum_ix Eg[iy][ix] W[ix][q],  W[ix][q] = w^(ix (q - L)) / L
//   column stage  Y[r][q]  = sum_iy V[r][iy] Z[iy][q],    V[r][iy] = w^(iy (r - L))
//
// with w = exp(2 pi i / N), so outputs come out in image pixel order (index L
// is the phase centre).  Phase vectors come in conjugate pairs: the column
// q' = N - q of W is the conjugate of column q, and likewise for the rows of V.
// Each stage therefore runs only over its base half (q < L, r < L): with the
// four real products
//   P1 = Re x . Re u,  P2 = Im x . Im u,  P3 = Re x . Im u,  P4 = Im x . Re u
// of the data x and the base phase vector u, the base output is
// (P1 - P2) + i (P3 + P4) and its partner's is (P1 + P2) + i (P4 - P3): half the
// matrix work of the plain complex product.  The two real self-conjugate
// vectors (q - L = -L, alternating signs, and q - L = 0, all ones) share the
// slot of index 0 as real and imaginary part, which gives them directly as
// P1 + i P4 and P3 + i P2.
//
// Operands are binary16 or bfloat16 (Eg rounded once when gridded, Z once
// between the stages, phase factors once from float64); every product
// accumulates in float32 (v_mfma_f32_16x16x32_{f16,bf16}).  The squared
// magnitudes accumulate as S = P1^2 + P2^2 + P3^2 + P4^2 and D = P3 P4 - P1 P2,
// so that base = S + 2 D and partner = S - 2 D (the shared slot takes S at
// half weight and its own D).
//
// One workgroup owns one (channel, time slice) and streams its frames through
// a three-deep pipeline.  Its waves have two roles:
//   * gather waves (2 at N = 64, 4 at N = 128) grid frame j - 1: each lane
//     walks its balanced slice of the cell-keyed program (no atomics) and
//     stores finished cells as 16-bit values;
//   * matrix waves (2 at N = 64, 8 at N = 128) ingest and calibrate frame j
//     (e = g E into LDS as float32, self power per antenna), and each runs one
//     row-stage panel of frame j - 2 (16 grid rows x 32 base columns) and one
//     column-stage tile of frame j - 3 (32 base rows x 32 columns).  The
//     column stage's phase factors stay in registers for the whole launch,
//     the row stage's are read from LDS.  Z goes through LDS transposed
//     (column-major), the layout the column stage reads; |Y|^2 accumulates in
//     registers.
// A wave issues its matrix products and its vector work (the pair
// combinations, the conversion of Z, the squared magnitudes) one after the
// other; two matrix waves per SIMD let one's vector work run beside the
// other's products, and the gather waves' latency-bound gridding runs beside
// both.  The samples, the grid and Z are double-buffered, so one
// barrier per frame orders every hand-over.  Every iteration runs both stages:
// the fill iterations transform the cleared buffers and add exact zeros.
// After the last frame the accumulators go through the same epilogue modes as
// the float32 fused kernel (per-slice partial, running sum, final image).
//
// MFMA operand layout (16x16x32): lane l supplies A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i < 8, and receives D[4 (l / 16) + j][l % 16] in
// accumulator j < 4.
//
// LDS rows are 2L + 8 sixteen-bit elements long (real parts, then imaginary
// parts): the 16-byte operand reads of consecutive rows then fall in different
// 16-byte bank groups.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class H>
__device__ __forceinline__ f32x4 mfma16(typename Vec<H>::v8 a, typename Vec<H>::v8 b, f32x4 c);

template <>
__device__ __forceinline__ f32x4 mfma16<_Float16>(Vec<_Float16>::v8 a, Vec<_Float16>::v8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f32x4 mfma16<__bf16>(Vec<__bf16>::v8 a, Vec<__bf16>::v8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int N>
struct MfmaShape {
  static constexpr int L = N / 2;
  static constexpr int NW = mfma_waves(N);          // matrix waves
  static constexpr int NG = mfma_gather_waves(N);   // gather waves
  static constexpr int NTG = NG * 64;               // gather lanes: the program's width
  static constexpr int NT = (NW + NG) * 64;         // threads per workgroup
  static constexpr int WPE = N == 128 ? 3 : 2;      // waves per SIMD the registers are sized for
  static constexpr int KS2 = L / 32;                // 32-deep steps over a contraction of L
  static constexpr int NRB = L / 32;                // base blocks of 32 (row-stage columns, column-stage rows)
  static constexpr int NIB = L / 32;                // row-stage blocks of 32 grid rows
  static constexpr int NQB = N / 32;                // column-stage blocks of 32 output columns
  static_assert(NW == 2 * NIB * NRB, "one row-stage panel (half a 32 x 32 tile) per matrix wave");
  static_assert(NW == NRB * NQB, "one column-stage tile per matrix wave");
  static constexpr int PITCH = 2 * L + 8;           // LDS row length, 16-bit elements
  static constexpr int EG = L * PITCH;              // one Eg [L][PITCH]: real parts at ix, imaginary at L + ix
  static constexpr int ZT = N * PITCH;              // one Zt [N][PITCH]: Zt[q][iy] = Re Z, Zt[q][L + iy] = Im Z
};

// LDS the program may take: at N = 128 one workgroup fills a compute unit (its
// registers allow no second one); at N = 64 two workgroups share one.
constexpr size_t mfma_prog_lds_limit(int N) { return N == 128 ? kMfmaLdsMax : kMfmaLdsMax / 2; }

// Program entries per gather lane that the gather waves keep in registers for
// the whole launch (with their tap values); a longer program is read every
// frame, from LDS when it fits there.
constexpr int mfma_prog_regs(int N) { return N == 128 ? 16 : 24; }

}  // namespace

size_t mfma_lds_bytes(int N, int n_taps, int n_ant, int prog_len, bool prog_in_lds) {
  const MfmaLayout m = mfma_layout(N, n_taps, n_ant);
  const size_t prog = prog_in_lds ? sizeof(GatherEntry) * static_cast<size_t>(prog_len) * (mfma_gather_waves(N) * 64) : 0;
  return static_cast<size_t>(m.prog) + prog;
}

// A program that fits the registers is read from global memory once, so it
// takes no LDS: at N = 64 three workgroups then share a compute unit.
bool mfma_prog_in_lds(int N, int n_taps, int n_ant, int prog_len) {
  return prog_len > mfma_prog_regs(N) && mfma_lds_bytes(N, n_taps, n_ant, prog_len, true) <= mfma_prog_lds_limit(N);
}

template <int N, class H, bool CI4>
__global__ __launch_bounds__((MfmaShape<N>::NT)) __attribute__((amdgpu_waves_per_eu(MfmaShape<N>::WPE)))
void mfma_kernel(MfmaArgs a) {
  using S = MfmaShape<N>;
  using V8 = typename Vec<H>::v8;
  using V4 = typename Vec<H>::v4;
  constexpr int NT = S::NT, NTG = S::NTG, L = S::L, KS2 = S::KS2, PITCH = S::PITCH;
  extern __shared__ uint4 lds_mfma[];
  __shared__ double Atot[kMaxTypesDev];
  __shared__ double pw_part[S::NW][kMaxTypesDev];   // self power per matrix wave and table type
  char* lds = reinterpret_cast<char*>(lds_mfma);
  const MfmaLayout lay = mfma_layout(N, a.n_taps, a.n_ant);
  float2* K = reinterpret_cast<float2*>(lds + lay.k);   // [n_taps]
  H* Eg = reinterpret_cast<H*>(lds + lay.eg);           // [2][EG]
  H* Zt = reinterpret_cast<H*>(lds + lay.zt);           // [2][ZT]
  float2* gl = reinterpret_cast<float2*>(lds + lay.gl); // [n_ant]
  int* ty = reinterpret_cast<int*>(lds + lay.ty);       // [n_ant]
  // gather program [prog_len][NTG], copied into LDS when it fits
  GatherEntry* lprog = reinterpret_cast<GatherEntry*>(lds + lay.prog);

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, uniform per wave
  const int item = blockIdx.x;
  if (item >= a.n_chan * a.slices) return;
  const int c = item % a.n_chan;
  const int slice = item / a.n_chan;

  // Both grids and both row-stage outputs cleared once: grid cells without
  // antennas are never written, and the pipeline's fill iterations transform
  // these zeros (an exact no-op for the accumulators).  Eg and Zt are adjacent.
  static_assert((2 * S::EG * 2) % 16 == 0 && (2 * S::ZT * 2) % 16 == 0, "buffers of whole 16-byte words");
  for (int i = tid; i < 2 * (S::EG + S::ZT) * 2 / 16; i += NT) reinterpret_cast<uint4*>(Eg)[i] = make_uint4(0u, 0u, 0u, 0u);
  for (int i = tid; i < a.n_taps; i += NT) K[i] = a.ktab[i];
  for (int i = tid; i < a.n_ant; i += NT) {
    ty[i] = a.ant_type[i];
    gl[i] = a.gains ? a.gains[static_cast<size_t>(c) * a.n_ant + i] : make_float2(1.f, 0.f);
  }
  if (tid < 2) reinterpret_cast<float2*>(lds + lay.e + tid * lay.e_stride)[a.n_ant] = make_float2(0.f, 0.f);
  {
    // the row stage's phase-factor operands (stage 0 of the table)
    constexpr int n_wt = S::NRB * 2 * KS2 * 2 * 64;   // 16-byte operands
    const uint4* src = reinterpret_cast<const uint4*>(a.dft);
    for (int i = tid; i < n_wt; i += NT) reinterpret_cast<uint4*>(lds + lay.wt)[i] = src[i];
  }
  if (a.prog_in_lds)
    for (int i = tid; i < a.prog_len * NTG; i += NT) lprog[i] = a.prog[i];

  const int64_t T = a.n_time;
  const int64_t t0 = slice * T / a.slices, t1 = (slice + 1) * T / a.slices;
  const int64_t nf = t1 - t0;
  // iteration j: matrix waves ingest frame j and run the row stage of frame
  // j - 2 and the column stage of frame j - 3; gather waves grid frame j - 1
  const int64_t n_iter = nf > 0 ? nf + 3 : 0;
  const int row = lane & 31, half = lane >> 5;
  __syncthreads();   // tables in LDS

  if (w < S::NW) {
    // ---- matrix waves ----
    // row-stage panel: grid rows 32 ib + 16 pm .. +16, base columns 32 qb .. +32
    const int pm = w % 2, ib = (w / 2) % S::NIB, qb = (w / 2) / S::NIB;
    // column-stage tile: base rows 32 rb .. +32, output columns 32 qc .. +32
    const int rb = w / S::NQB, qc = w % S::NQB;
    const int l16 = lane & 15, g16 = lane >> 4;
    // Phase factors (real, imaginary part): V, the column stage's A operand per
    // 16-row half, is resident in registers for the whole launch; W, the row
    // stage's B operand per 16-column half, is read from LDS one step at a
    // time (it is used once per frame, and registers are what bound this role).
    V8 vc[2][KS2], vd[2][KS2];
    {
      const V8* src = reinterpret_cast<const V8*>(a.dft);
      auto at = [&](int st, int blk, int hf, int ks, int part) {
        return src[((((st * S::NRB + blk) * 2 + hf) * KS2 + ks) * 2 + part) * 64 + lane];
      };
#pragma unroll
      for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int ks = 0; ks < KS2; ++ks) {
          vc[hf][ks] = at(1, rb, hf, ks, 0);
          vd[hf][ks] = at(1, rb, hf, ks, 1);
        }
    }
    const V8* wt = reinterpret_cast<const V8*>(lds + lay.wt);
    auto w_op = [&](int hf, int ks, int part) { return wt[(((qb * 2 + hf) * KS2 + ks) * 2 + part) * 64 + lane]; };
    // index 0 of base block 0 is the shared slot of the two real phase vectors
    const bool sp_row = rb == 0 && g16 == 0;   // column stage: accumulator (half 0, j 0) is row r = 0
    const bool sp_col = qb == 0 && l16 == 0;   // row stage: this lane's half-0 column is q = 0
    const float s_col = sp_col ? 0.f : 1.f;
    // S in acc_s, D in acc_d per column-stage half h and accumulator e = 4 m + j:
    // base = S + 2 D, partner = S - 2 D.  For the shared slot S is taken at half
    // weight and D as (P1^2 + P4^2 - P2^2 - P3^2) / 4, which makes the same two
    // formulas give |P1 + i P4|^2 and |P3 + i P2|^2.
    float acc_s[2][8], acc_d[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int e = 0; e < 8; ++e) acc_s[h][e] = acc_d[h][e] = 0.f;

    // Ingest and calibration of frame j (e = g E into LDS as float32, self
    // power per antenna), one antenna per matrix lane and prefetch slot.  Raw
    // samples of the next frame are loaded one iteration ahead, so the HBM
    // latency is hidden behind this iteration's matrix work; antennas beyond
    // the prefetch slots are loaded when used.  Per-lane self-power sums are
    // float32 (this path's error budget is set by its 16-bit operands); lanes
    // are combined in float64.
    constexpr int NI = S::NW * 64, kPrefetch = N == 128 ? 1 : 2;
    const size_t frame_stride = static_cast<size_t>(a.n_chan) * a.n_ant;
    float2 raw[kPrefetch];
    float pws[kPrefetch];
#pragma unroll
    for (int q = 0; q < kPrefetch; ++q) pws[q] = 0.f;
    float pwt[kMaxTypesDev] = {0.f, 0.f, 0.f, 0.f};
    auto load_raw = [&](int64_t t) {
      const size_t base = static_cast<size_t>(t) * frame_stride + static_cast<size_t>(c) * a.n_ant;
#pragma unroll
      for (int q = 0; q < kPrefetch; ++q) {
        const int i = tid + q * NI;
        if (i < a.n_ant) raw[q] = load_sample(a.E, base + i, CI4);
      }
    };
    auto ingest = [&](int64_t t, float2* e) {
#pragma unroll
      for (int q = 0; q < kPrefetch; ++q) {
        const int i = tid + q * NI;
        if (i < a.n_ant) {
          const float2 v = c_mul(gl[i], raw[q]);
          e[i] = v;
          pws[q] += fmaf(v.x, v.x, v.y * v.y);
        }
      }
      const size_t base = static_cast<size_t>(t) * frame_stride + static_cast<size_t>(c) * a.n_ant;
      for (int i = tid + kPrefetch * NI; i < a.n_ant; i += NI) {
        const float2 v = c_mul(gl[i], load_sample(a.E, base + i, CI4));
        e[i] = v;
        const float p = fmaf(v.x, v.x, v.y * v.y);
        const int tp = ty[i];
#pragma unroll
        for (int q = 0; q < kMaxTypesDev; ++q) pwt[q] += (tp == q) ? p : 0.f;
      }
    };
    if (nf > 0) load_raw(t0);

    for (int64_t j = 0; j < n_iter; ++j) {
      if (j < nf) ingest(t0 + j, reinterpret_cast<float2*>(lds + lay.e + (j & 1) * lay.e_stride));
      // row stage of frame j - 2, then column stage of frame j - 3
      const H* eg = Eg + ((j - 2) & 1) * S::EG;
      H* zw = Zt + ((j - 2) & 1) * S::ZT;
      const H* zr = Zt + ((j - 3) & 1) * S::ZT;
      // operands of the three panels: [panel][k-step][real, imaginary part]
      auto src = [&](int p, int ks, int part) {
        const H* base = p == 0 ? eg + (32 * ib + 16 * pm + l16) * PITCH : zr + (32 * qc + 16 * (p - 1) + l16) * PITCH;
        return reinterpret_cast<const V8*>(base + part * L + 32 * ks + 8 * g16);
      };
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        // this panel's operands (the other matrix wave on the SIMD covers their latency)
        V8 op[KS2][2];
#pragma unroll
        for (int ks = 0; ks < KS2; ++ks)
#pragma unroll
          for (int part = 0; part < 2; ++part) op[ks][part] = *src(p, ks, part);
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
          // one 16-wide half of the panel: four products over the contraction
          f32x4 Q[4];
#pragma unroll
          for (int ks = 0; ks < KS2; ++ks) {
            const V8 xa = op[ks][0], xb = op[ks][1];
            const f32x4 z = {};
            if (p == 0) {   // row stage: A = Eg (real, imaginary part), B = W half hf
              const V8 wr = w_op(hf, ks, 0), wi = w_op(hf, ks, 1);
              Q[0] = mfma16<H>(xa, wr, ks ? Q[0] : z);
              Q[1] = mfma16<H>(xb, wi, ks ? Q[1] : z);
              Q[2] = mfma16<H>(xa, wi, ks ? Q[2] : z);
              Q[3] = mfma16<H>(xb, wr, ks ? Q[3] : z);
            } else {        // column stage: A = V half hf, B = Z (real, imaginary part)
              Q[0] = mfma16<H>(vc[hf][ks], xa, ks ? Q[0] : z);
              Q[1] = mfma16<H>(vd[hf][ks], xb, ks ? Q[1] : z);
              Q[2] = mfma16<H>(vd[hf][ks], xa, ks ? Q[2] : z);
              Q[3] = mfma16<H>(vc[hf][ks], xb, ks ? Q[3] : z);
            }
          }
          if (p == 0) {
            // Z of grid rows iy = 32 ib + 16 pm + 4 g16 + (0..3): base column q
            // and its partner
            const int q = 32 * qb + 16 * hf + l16;
            const bool sp = hf == 0 && sp_col;
            const float sc = hf == 0 ? s_col : 1.f;
            const int qp = sp ? L : N - q;
            V4 br, bi, pr, pi;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              br[jj] = static_cast<H>(fmaf(-sc, Q[1][jj], Q[0][jj]));
              bi[jj] = static_cast<H>(fmaf(sc, Q[2][jj], Q[3][jj]));
              pr[jj] = static_cast<H>(sp ? Q[2][jj] : Q[0][jj] + Q[1][jj]);
              pi[jj] = static_cast<H>(sp ? Q[1][jj] : Q[3][jj] - Q[2][jj]);
            }
            const int iy = 32 * ib + 16 * pm + 4 * g16;
            *reinterpret_cast<V4*>(zw + q * PITCH + iy) = br;
            *reinterpret_cast<V4*>(zw + q * PITCH + L + iy) = bi;
            *reinterpret_cast<V4*>(zw + qp * PITCH + iy) = pr;
            *reinterpret_cast<V4*>(zw + qp * PITCH + L + iy) = pi;
          } else {
            const int h = p - 1;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const int e = 4 * hf + jj;
              if (e == 0) {
                const float sq = fmaf(Q[0][0], Q[0][0], fmaf(Q[1][0], Q[1][0], fmaf(Q[2][0], Q[2][0], Q[3][0] * Q[3][0])));
                const float d = fmaf(Q[2][0], Q[3][0], -Q[0][0] * Q[1][0]);
                const float ds = 0.25f * (fmaf(Q[0][0], Q[0][0], Q[3][0] * Q[3][0]) - fmaf(Q[1][0], Q[1][0], Q[2][0] * Q[2][0]));
                acc_s[h][0] = fmaf(sp_row ? 0.5f : 1.f, sq, acc_s[h][0]);
                acc_d[h][0] += sp_row ? ds : d;
              } else {
                acc_s[h][e] = fmaf(Q[0][jj], Q[0][jj], fmaf(Q[1][jj], Q[1][jj], fmaf(Q[2][jj], Q[2][jj], fmaf(Q[3][jj], Q[3][jj], acc_s[h][e]))));
                acc_d[h][e] = fmaf(Q[2][jj], Q[3][jj], fmaf(-Q[0][jj], Q[1][jj], acc_d[h][e]));
              }
            }
          }
        }
      }
      // the samples of frame j + 1, requested after this iteration's work
      if (j + 1 < nf) load_raw(t0 + j + 1);
      __syncthreads();
    }
    {
      // self power per table type: lanes in float64, then one partial per wave
      double pw[kMaxTypesDev];
#pragma unroll
      for (int q = 0; q < kMaxTypesDev; ++q) pw[q] = pwt[q];
#pragma unroll
      for (int q = 0; q < kPrefetch; ++q) {
        const int i = tid + q * NI;
        if (i < a.n_ant) {
          const int tp = ty[i];
#pragma unroll
          for (int p = 0; p < kMaxTypesDev; ++p) pw[p] += (tp == p) ? static_cast<double>(pws[q]) : 0.0;
        }
      }
#pragma unroll
      for (int p = 0; p < kMaxTypesDev; ++p) {
        double x = pw[p];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) pw_part[w][p] = x;
      }
    }
    __syncthreads();   // self-power partials of the matrix waves are in LDS
    if (tid < kMaxTypesDev) {
      double s = 0.0;
      for (int g = 0; g < S::NW; ++g) s += pw_part[g][tid];
      Atot[tid] = s;
    }
    __syncthreads();   // Atot complete (the gather waves take part in every barrier)

    // epilogue: the row stage carried a factor 1 / L, so |Y|^2 is scaled back by L^2 (exact)
    const size_t img_stride = static_cast<size_t>(N) * N;
    constexpr float kBack = static_cast<float>(L) * static_cast<float>(L);
    auto put = [&](int r, int q, float v) {
      const size_t pix = static_cast<size_t>(r) * N + q;
      const float s = v * kBack;
      if (a.mode == kModePartial) {
        a.out[(static_cast<size_t>(slice) * a.n_chan + c) * img_stride + pix] = s;
      } else if (a.mode == kModeAccum) {
        a.out[static_cast<size_t>(c) * img_stride + pix] += s;
      } else {
        double x = s;
        if (a.subtract)
          for (int p = 0; p < a.n_types; ++p) x -= Atot[p] * a.Pp[p * img_stride + pix];
        a.out[static_cast<size_t>(c) * img_stride + pix] = static_cast<float>(x * a.scale);
      }
    };
    // both 64-byte halves of an image row's 128-byte line go out back to back
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = 32 * rb + 16 * (e / 4) + 4 * g16 + (e % 4);
      const int rp = r == 0 ? L : N - r;
#pragma unroll
      for (int h = 0; h < 2; ++h) put(r, 32 * qc + 16 * h + l16, fmaf(2.f, acc_d[h][e], acc_s[h][e]));
#pragma unroll
      for (int h = 0; h < 2; ++h) put(rp, 32 * qc + 16 * h + l16, fmaf(-2.f, acc_d[h][e], acc_s[h][e]));
    }
    if (tid < a.n_types) {
      if (a.mode == kModePartial) {
        a.outA[(static_cast<size_t>(slice) * a.n_chan + c) * a.n_types + tid] = Atot[tid];
      } else if (a.mode == kModeAccum) {
        a.outA[static_cast<size_t>(c) * a.n_types + tid] += Atot[tid];
      }
    }
  } else {
    // ---- gather waves ----
    const int gt = tid - S::NW * 64;   // gather lane, 0 .. NTG - 1 (the matrix waves come first)
    // Gather-gridding of frame j - 1: each lane walks its balanced slice of the
    // cell-keyed program (no atomics) and stores finished cells as 16-bit values.
    // entry: x = byte offsets of e[ant] (low half, buffer 0) and K[tap] (high
    // half), y = byte address of the finished cell's real part in grid 0, or 0.
    // The program pointer is either LDS or global memory, never a select of
    // the two: a pointer of unknown address space compiles to flat loads, whose
    // waits also drain the (in-order) global-load counter.
    auto gather = [&](const GatherEntry* prog, int eoff, int goff) {
      float2 g = make_float2(0.f, 0.f);
      auto step = [&](GatherEntry en) {
        const float2 ev = *reinterpret_cast<const float2*>(lds + eoff + (en.x & 0xFFFFu));
        const float2 kv = *reinterpret_cast<const float2*>(lds + (en.x >> 16));
        g.x = fmaf(ev.x, kv.x, fmaf(-ev.y, kv.y, g.x));
        g.y = fmaf(ev.x, kv.y, fmaf(ev.y, kv.x, g.y));
        if (en.y != 0u) {
          H* cell = reinterpret_cast<H*>(lds + goff + en.y);
          cell[0] = static_cast<H>(g.x);
          cell[L] = static_cast<H>(g.y);
          g = make_float2(0.f, 0.f);
        }
      };
      int k = 0;
      for (; k + 4 <= a.prog_len; k += 4) {
        GatherEntry en[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) en[i] = prog[static_cast<size_t>(k + i) * NTG];
#pragma unroll
        for (int i = 0; i < 4; ++i) step(en[i]);
      }
      for (; k < a.prog_len; ++k) step(prog[static_cast<size_t>(k) * NTG]);
    };

    // The program does not change from frame to frame: when it is short
    // enough, each lane keeps its entries and their tap values in registers,
    // and a frame costs one batch of sample reads from LDS.
    constexpr int kProgRegs = mfma_prog_regs(N);
    const bool prog_in_regs = a.prog_len <= kProgRegs;
    uint32_t r_e[kProgRegs], r_cell[kProgRegs];
    float2 r_k[kProgRegs];
    if (prog_in_regs) {
#pragma unroll
      for (int k = 0; k < kProgRegs; ++k) {
        GatherEntry en = {static_cast<uint32_t>(lay.e + 8 * a.n_ant) | (static_cast<uint32_t>(lay.k) << 16), 0u};
        if (k < a.prog_len) en = a.prog_in_lds ? lprog[k * NTG + gt] : a.prog[static_cast<size_t>(k) * NTG + gt];
        r_e[k] = en.x & 0xFFFFu;
        r_cell[k] = en.y;
        r_k[k] = *reinterpret_cast<const float2*>(lds + (en.x >> 16));
      }
    }
    // Entries past the program's end are padding (the zero sample, no store),
    // so the loops have no trip-count branches; a shorter copy covers the
    // first 3/4 of the slots, for programs that fit there.
    constexpr int kShort = kProgRegs * 3 / 4;
    auto gather_regs = [&](auto count, int eoff, int goff) {
      constexpr int K = decltype(count)::value;
      float2 ev[K];
#pragma unroll
      for (int k = 0; k < K; ++k) ev[k] = *reinterpret_cast<const float2*>(lds + eoff + r_e[k]);
      float2 g = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        g.x = fmaf(ev[k].x, r_k[k].x, fmaf(-ev[k].y, r_k[k].y, g.x));
        g.y = fmaf(ev[k].x, r_k[k].y, fmaf(ev[k].y, r_k[k].x, g.y));
        if (r_cell[k] != 0u) {
          H* cell = reinterpret_cast<H*>(lds + goff + r_cell[k]);
          cell[0] = static_cast<H>(g.x);
          cell[L] = static_cast<H>(g.y);
          g = make_float2(0.f, 0.f);
        }
      }
    };

    for (int64_t j = 0; j < n_iter; ++j) {
      if (j >= 1 && j - 1 < nf) {
        const int eoff = ((j - 1) & 1) * lay.e_stride, goff = ((j - 1) & 1) * lay.eg_stride;
        if (a.prog_len <= kShort)
          gather_regs(std::integral_constant<int, kShort>(), eoff, goff);
        else if (prog_in_regs)
          gather_regs(std::integral_constant<int, kProgRegs>(), eoff, goff);
        else if (a.prog_in_lds)
          gather(lprog + gt, eoff, goff);
        else
          gather(a.prog + gt, eoff, goff);
      }
      __syncthreads();
    }
    __syncthreads();   // self-power partials visible to the matrix waves
    __syncthreads();   // matrix waves have read them (Atot)
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
