// The per-frame transform of the fused and staged kernels: the zero-padded
// 2-D DFT of one channel-frame, restricted to the output columns
// q = SX * m + w of one workgroup, staged in LDS (Sec. 3, spatial Fourier
// transform; zero padding to twice the aperture per axis, Sec. 6.1).
//
// Layout in LDS: the folded aperture grid G[iy][n'] (iy < L, n' < M, row
// pitch M + 1 complex elements), where
//     G[iy][n'] = sum_j exp(+2 pi i j w / SX) Eg[iy][n' + j M]
// so that the output column q = SX m + w of row iy is
//     Z[iy][m] = sum_{n'} G[iy][n'] w_N^{n' w} w_M^{n' m}      (an M-point DFT),
// and the output pixel (r, q) is Y[r][q] = sum_{iy < L} Z[iy][m] w_N^{iy r}
// (an N-point DFT with the upper half of its inputs zero).
//
// Rows are transformed in place by the waves that own them (radix PR over a
// stride-QR decimation, then radix QR), columns in place by the waves that own
// them in two half-rounds s = 0, 1 that produce the output rows r = q1 + PC q2
// with q1 = 2 j + s; each half-round fits back into the L column slots.  Only
// wave-level ordering is needed inside a stage; the caller separates stages
// with workgroup barriers.
#pragma once

#include "dft.h"
#include "shape.h"

namespace moff {

// Order LDS accesses of one wave: the LDS unit executes a wave's DS
// instructions in issue order, so a compiler-level fence is enough.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Lane mapping.  Every line (row or column) is transformed by LP lanes of one
// wave that sit 64/LP apart (lane = line_in_step + (64/LP) sub), so each group of
// 16 consecutive lanes touches 16 different lines at the same position.  With a
// row pitch of M + 1 (odd) every 8-byte LDS access of the transform then hits 16
// distinct banks per 16-lane group -- the unit in which gfx950 serves 64-bit LDS
// accesses -- and every address is a per-lane base plus a compile-time offset.
template <int N_, int V_ = 0>
struct FT {
  static constexpr FrameShape S = frame_shape(N_, V_);
  static constexpr int N = N_, NT = S.NT, SX = S.SX, M = N / SX, L = N / 2, NW = NT / 64;
  static constexpr int PR = S.PR, QR = S.QR, PC = S.PC, QC = S.QC;
  static constexpr int NZR = L < M ? L : M;
  static constexpr int PRNZ = NZR / QR;          // nonzero inputs of the row pass A
  static constexpr int LPR = row_lanes(S);       // lanes per row
  static constexpr int RPW = 64 / LPR;           // rows per wave per step
  static constexpr int JAR = QR / LPR;           // row pass-A jobs per lane
  static constexpr int JBR = PR / LPR;           // row pass-B jobs per lane
  static constexpr int RSTEPS = (L + NW * RPW - 1) / (NW * RPW);
  static constexpr bool RGUARD = (L % (NW * RPW)) != 0;
  static constexpr int PH = PC / 2;              // column pass-A length per half-round
  static constexpr int LPC = cmin(4, cmin(QC, PH));  // lanes per column
  static constexpr int CPW = 64 / LPC;           // columns per wave per step
  static constexpr int JA = QC / LPC;            // column pass-A jobs per lane
  static constexpr int JB = PH / LPC;            // column pass-B jobs per lane per half-round
  static constexpr int CSTEPS = (M + NW * CPW - 1) / (NW * CPW);
  static constexpr bool CGUARD = (M % (NW * CPW)) != 0;
  static constexpr int P = M + 1;                // LDS row pitch of the folded grid
  static constexpr int GRID = L * P;             // folded grid, complex elements
  static constexpr int TWR = PR * QR;            // row twiddle table [q1][n2]
  static constexpr int TWC = PC * QC;            // column twiddle table [q1][n2]
  static constexpr int NACC = CSTEPS * 2 * JB * QC;
  static_assert(PR * QR == M && PC * QC == N, "bad factorisation");
  static_assert(PH * QC == L, "column half-round must fill the L slots");
  static_assert(QR % LPR == 0 && PR % LPR == 0 && QC % LPC == 0 && PH % LPC == 0, "bad lanes");
  static_assert(NZR % QR == 0, "row pruning must align with the decimation");
};

// Per-workgroup twiddle tables (LDS), built once per launch from w_N^k:
//   twr[q1 * QR + n2] = w_M^{n2 q1} w_N^{n2 w}   (row pass-A outputs; the second
//                        factor is the part of the fold twiddle w_N^{n' w},
//                        n' = QR n1 + n2, that does not depend on n1)
//   twc[q1 * QC + n2] = w_N^{n2 q1}               (column pass-A outputs)
template <int N, int V>
__device__ __forceinline__ void build_twiddles(const float2* __restrict__ tw_global, int w, float2* twr, float2* twc) {
  using C = FT<N, V>;
  for (int i = threadIdx.x; i < C::TWR; i += C::NT) {
    const int q1 = i / C::QR, n2 = i % C::QR;
    twr[i] = tw_global[(C::SX * n2 * q1 + n2 * w) & (N - 1)];
  }
  for (int i = threadIdx.x; i < C::TWC; i += C::NT) {
    const int q1 = i / C::QC, n2 = i % C::QC;
    twc[i] = tw_global[(n2 * q1) & (N - 1)];
  }
}

// The n1-dependent part of the fold twiddle, w_N^{QR n1 w}, for this workgroup.
template <int N, int V>
__device__ __forceinline__ void fold_factors(const float2* __restrict__ tw_global, int w, float2 (&fin)[FT<N, V>::PRNZ]) {
  using C = FT<N, V>;
#pragma unroll
  for (int n1 = 0; n1 < C::PRNZ; ++n1) fin[n1] = tw_global[(C::QR * n1 * w) & (N - 1)];
}

// Row stage: Z[iy][m] = sum_{n'} G[iy][n'] w_N^{n' w} w_M^{n' m}, in place.
// Pass A (job n2): radix-PR DFT over the stride-QR decimation n' = QR n1 + n2,
// result (q1, n2) stored at q1 QR + n2; pass B (job q1): radix-QR DFT over n2,
// result stored at m = q1 + PR q2.
template <int N, int V>
__device__ __forceinline__ void row_stage(float2* G, const float2* twr, const float2 (&fin)[FT<N, V>::PRNZ]) {
  using C = FT<N, V>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / C::RPW;
  const float2* twrl = twr + sub;   // twrl[q1 QR + LPR ja] = twr[q1 QR + n2]
#pragma unroll
  for (int rs = 0; rs < C::RSTEPS; ++rs) {
    const int row = stage_row(C::S, rs, wave, lane % C::RPW);
    if (C::RGUARD && row >= C::L) continue;
    float2* R = G + row * C::P;
    float2 x[C::JAR][C::PR];
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja)
#pragma unroll
      for (int n1 = 0; n1 < C::PRNZ; ++n1) {
        x[ja][n1] = R[sub + C::LPR * ja + C::QR * n1];
        if constexpr (C::SX > 1) x[ja][n1] = c_mul(x[ja][n1], fin[n1]);
      }
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja) {
      dft_pruned<C::PR, C::PRNZ>(x[ja]);
#pragma unroll
      for (int q1 = (C::SX > 1 ? 0 : 1); q1 < C::PR; ++q1) x[ja][q1] = c_mul(x[ja][q1], twrl[q1 * C::QR + C::LPR * ja]);
    }
    wave_sync();
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja)
#pragma unroll
      for (int q1 = 0; q1 < C::PR; ++q1) R[sub + C::LPR * ja + q1 * C::QR] = x[ja][q1];
    wave_sync();
    float2 y[C::JBR][C::QR];
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb)
#pragma unroll
      for (int k = 0; k < C::QR; ++k) y[jb][k] = R[(sub + C::LPR * jb) * C::QR + k];
    wave_sync();
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb) {
      Dft<C::QR>::run(y[jb]);
#pragma unroll
      for (int q2 = 0; q2 < C::QR; ++q2) R[sub + C::LPR * jb + C::PR * q2] = y[jb][q2];
    }
    wave_sync();
  }
}

// Row stage of column class W known at compile time: the same transform as
// row_stage, with the fold factor of input n1, w_N^{QR n1 W} =
// exp(+2 pi i n1 W / (N / QR)), applied as a constant rotation (none for
// class 0, whose per-lane fold twiddle is 1 as well).
template <int N, int V, int W>
__device__ __forceinline__ void row_stage_w(float2* G, const float2* twr) {
  using C = FT<N, V>;
  constexpr bool kFold = C::SX > 1 && W != 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / C::RPW;
  const float2* twrl = twr + sub;   // twrl[q1 QR + LPR ja] = twr[q1 QR + n2]
#pragma unroll
  for (int rs = 0; rs < C::RSTEPS; ++rs) {
    const int row = stage_row(C::S, rs, wave, lane % C::RPW);
    if (C::RGUARD && row >= C::L) continue;
    float2* R = G + row * C::P;
    float2 x[C::JAR][C::PR];
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja)
      static_for<0, C::PRNZ>([&](auto nc) {
        constexpr int n1 = decltype(nc)::value;
        x[ja][n1] = R[sub + C::LPR * ja + C::QR * n1];
        if constexpr (kFold) x[ja][n1] = rot<N / C::QR, n1 * W>(x[ja][n1]);
      });
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja) {
      dft_pruned<C::PR, C::PRNZ>(x[ja]);
#pragma unroll
      for (int q1 = (kFold ? 0 : 1); q1 < C::PR; ++q1) x[ja][q1] = c_mul(x[ja][q1], twrl[q1 * C::QR + C::LPR * ja]);
    }
    wave_sync();
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja)
#pragma unroll
      for (int q1 = 0; q1 < C::PR; ++q1) R[sub + C::LPR * ja + q1 * C::QR] = x[ja][q1];
    wave_sync();
    float2 y[C::JBR][C::QR];
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb)
#pragma unroll
      for (int k = 0; k < C::QR; ++k) y[jb][k] = R[(sub + C::LPR * jb) * C::QR + k];
    wave_sync();
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb) {
      Dft<C::QR>::run(y[jb]);
#pragma unroll
      for (int q2 = 0; q2 < C::QR; ++q2) R[sub + C::LPR * jb + C::PR * q2] = y[jb][q2];
    }
    wave_sync();
  }
}

// Column stage: Y[r][m] = sum_{iy < L} Z[iy][m] w_N^{iy r} for r < N, in place,
// handing every output to sink(acc_index, r, m, value) with acc_index in [0, NACC).
// Pass A (job n2): the pruned radix-PC DFT over rows QC n1 + n2, split by the
// parity s of its output q1 = 2 j + s into two half-rounds whose PH outputs are
// stored at rows j QC + n2; pass B (job j): radix-QC DFT over n2, output row
// r = q1 + PC q2.
template <int N, int V, class Sink>
__device__ __forceinline__ void col_stage(float2* G, const float2* twc, Sink&& sink) {
  using C = FT<N, V>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / C::CPW;
  const float2* twl = twc + sub;   // twl[q1 QC + LPC ja] = twc[q1 QC + n2]
#pragma unroll
  for (int cs = 0; cs < C::CSTEPS; ++cs) {
    const int col = (cs * C::NW + wave) * C::CPW + lane % C::CPW;
    if (C::CGUARD && col >= C::M) continue;
    float2* Zc = G + col + sub * C::P;     // row `sub` of this column
    float2 z[C::JA][C::PH];
#pragma unroll
    for (int ja = 0; ja < C::JA; ++ja)
#pragma unroll
      for (int n1 = 0; n1 < C::PH; ++n1) z[ja][n1] = Zc[(C::LPC * ja + C::QC * n1) * C::P];
    wave_sync();
    static_for<0, 2>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
#pragma unroll
      for (int ja = 0; ja < C::JA; ++ja) {
        float2 u[C::PH];
        static_for<0, C::PH>([&](auto nc) {
          constexpr int n1 = decltype(nc)::value;
          if constexpr (s == 0) u[n1] = z[ja][n1];
          else u[n1] = rot<C::PC, n1>(z[ja][n1]);
        });
        Dft<C::PH>::run(u);
#pragma unroll
        for (int j = 0; j < C::PH; ++j) {
          const int q1 = 2 * j + s;
          if (q1 != 0) u[j] = c_mul(u[j], twl[q1 * C::QC + C::LPC * ja]);
          Zc[(C::LPC * ja + j * C::QC) * C::P] = u[j];
        }
      }
      wave_sync();
      float2 v[C::JB][C::QC];
      const float2* Zb = G + col + sub * C::QC * C::P;   // row (sub QC) of this column
#pragma unroll
      for (int jb = 0; jb < C::JB; ++jb)
#pragma unroll
        for (int k = 0; k < C::QC; ++k) v[jb][k] = Zb[(C::LPC * jb * C::QC + k) * C::P];
      wave_sync();
#pragma unroll
      for (int jb = 0; jb < C::JB; ++jb) {
        const int j = sub + C::LPC * jb;
        Dft<C::QC>::run(v[jb]);
#pragma unroll
        for (int q2 = 0; q2 < C::QC; ++q2) {
          const int r = 2 * j + s + C::PC * q2;
          sink(((cs * 2 + s) * C::JB + jb) * C::QC + q2, r, col, v[jb][q2]);
        }
      }
    });
  }
}

// Output pixel coordinates (r, m) of accumulator `idx` for thread `tid`; the
// same mapping col_stage hands to its sink.
template <int N, int V>
__host__ __device__ __forceinline__ void acc_pixel_of(int tid, int idx, int& r, int& col) {
  using C = FT<N, V>;
  const int lane = tid & 63, wave = tid >> 6;
  const int q2 = idx % C::QC;
  const int jb = (idx / C::QC) % C::JB;
  const int s = (idx / (C::QC * C::JB)) % 2;
  const int cs = idx / (C::QC * C::JB * 2);
  const int j = lane / C::CPW + C::LPC * jb;
  col = (cs * C::NW + wave) * C::CPW + lane % C::CPW;
  r = 2 * j + s + C::PC * q2;
}

// The same for this lane.
template <int N, int V>
__device__ __forceinline__ void acc_pixel(int idx, int& r, int& col) {
  using C = FT<N, V>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q2 = idx % C::QC;
  const int jb = (idx / C::QC) % C::JB;
  const int s = (idx / (C::QC * C::JB)) % 2;
  const int cs = idx / (C::QC * C::JB * 2);
  const int j = lane / C::CPW + C::LPC * jb;
  col = (cs * C::NW + wave) * C::CPW + lane % C::CPW;
  r = 2 * j + s + C::PC * q2;
}

// ---------------------------------------------------------------------------
// Adjoint (transpose) of the frame transform, for gradients.  With F the
// forward map from the folded grid G[iy][n'] (n' < NZR) to the workgroup's
// output pixels Y[r][m], these compute F^H: exponents are negated, twiddles
// conjugated, and the zero-input half of each forward DFT becomes an
// output-pruned inverse DFT.
// ---------------------------------------------------------------------------

// Column stage adjoint: from values src(acc_index, r, m) at this lane's pixels
// (the pixels col_stage hands to its sink) to Z'[iy][m] = sum_r Y'[r][m] w_N^{-iy r}
// for iy < L, written in place into G.
template <int N, int V, class Source>
__device__ __forceinline__ void col_stage_adjoint(float2* G, const float2* twc, Source&& src) {
  using C = FT<N, V>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / C::CPW;
  const float2* twb = twc + 2 * sub * C::QC;   // twb[(2 LPC jb + s) QC + n2] = twc[q1 QC + n2]
#pragma unroll
  for (int cs = 0; cs < C::CSTEPS; ++cs) {
    const int col = (cs * C::NW + wave) * C::CPW + lane % C::CPW;
    if (C::CGUARD && col >= C::M) continue;
    float2* Zc = G + col + sub * C::P;            // row `sub` of this column
    float2* Zb = G + col + sub * C::QC * C::P;    // row (sub QC) of this column
    float2 xacc[C::JA][C::PH];
#pragma unroll
    for (int ja = 0; ja < C::JA; ++ja)
#pragma unroll
      for (int n1 = 0; n1 < C::PH; ++n1) xacc[ja][n1] = make_float2(0.f, 0.f);
    static_for<0, 2>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      // pass B^H (job j): inverse radix-QC over q2, conjugate twiddles, rows j QC + n2
#pragma unroll
      for (int jb = 0; jb < C::JB; ++jb) {
        const int j = sub + C::LPC * jb;
        const int q1 = 2 * j + s;
        float2 v[C::QC];
#pragma unroll
        for (int q2 = 0; q2 < C::QC; ++q2)
          v[q2] = src(((cs * 2 + s) * C::JB + jb) * C::QC + q2, q1 + C::PC * q2, col);
        idft<C::QC>(v);
#pragma unroll
        for (int n2 = 0; n2 < C::QC; ++n2) {
          if (q1 != 0) v[n2] = c_mul_conj(v[n2], twb[(2 * C::LPC * jb + s) * C::QC + n2]);
          Zb[(C::LPC * jb * C::QC + n2) * C::P] = v[n2];
        }
      }
      wave_sync();
      // pass A^H (job n2), half-round s: inverse radix-PH over j, times w_PC^{-n1 s}
#pragma unroll
      for (int ja = 0; ja < C::JA; ++ja) {
        float2 u[C::PH];
#pragma unroll
        for (int j = 0; j < C::PH; ++j) u[j] = Zc[(C::LPC * ja + j * C::QC) * C::P];
        idft<C::PH>(u);
        static_for<0, C::PH>([&](auto nc) {
          constexpr int n1 = decltype(nc)::value;
          const float2 t = (s == 0) ? u[n1] : rot<C::PC, -n1>(u[n1]);
          xacc[ja][n1] = c_add(xacc[ja][n1], t);
        });
      }
      wave_sync();
    });
#pragma unroll
    for (int ja = 0; ja < C::JA; ++ja)
#pragma unroll
      for (int n1 = 0; n1 < C::PH; ++n1) Zc[(C::LPC * ja + C::QC * n1) * C::P] = xacc[ja][n1];
    wave_sync();
  }
}

// Column stage followed by its adjoint, column by column in place: the forward
// pruned column DFT, each output pixel scaled by its sensitivity, and the
// adjoint back to Z'[iy][m] for iy < L.  The same as col_stage into a buffer,
// a pixel-wise product and col_stage_adjoint from it, without holding the
// column's outputs.  The sensitivities of pass-B job (cs, s, jb) -- the QC
// pixels col_stage hands to its sink with accumulator indices
// ((cs * 2 + s) * JB + jb) * QC + q2 -- come from rload(cs, s, jb, r), called
// before that job's forward transform so that a load from memory overlaps it.
template <int N, int V, class RLoad>
__device__ __forceinline__ void col_stage_roundtrip(float2* G, const float2* twc, RLoad&& rload) {
  using C = FT<N, V>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / C::CPW;
  const float2* twb = twc + 2 * sub * C::QC;   // twb[(2 LPC jb + s) QC + n2] = twc[q1 QC + n2]
  const float2* twl = twc + sub;   // twl[q1 QC + LPC ja] = twc[q1 QC + n2]
#pragma unroll
  for (int cs = 0; cs < C::CSTEPS; ++cs) {
    const int col = (cs * C::NW + wave) * C::CPW + lane % C::CPW;
    if (C::CGUARD && col >= C::M) continue;
    float2* Zc = G + col + sub * C::P;            // row `sub` of this column
    float2* Zb = G + col + sub * C::QC * C::P;    // row (sub QC) of this column
    float2 z[C::JA][C::PH], xacc[C::JA][C::PH];
#pragma unroll
    for (int ja = 0; ja < C::JA; ++ja)
#pragma unroll
      for (int n1 = 0; n1 < C::PH; ++n1) {
        z[ja][n1] = Zc[(C::LPC * ja + C::QC * n1) * C::P];
        xacc[ja][n1] = make_float2(0.f, 0.f);
      }
    wave_sync();
    static_for<0, 2>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      // forward pass A, half-round s
#pragma unroll
      for (int ja = 0; ja < C::JA; ++ja) {
        float2 u[C::PH];
        static_for<0, C::PH>([&](auto nc) {
          constexpr int n1 = decltype(nc)::value;
          if constexpr (s == 0) u[n1] = z[ja][n1];
          else u[n1] = rot<C::PC, n1>(z[ja][n1]);
        });
        Dft<C::PH>::run(u);
#pragma unroll
        for (int j = 0; j < C::PH; ++j) {
          const int q1 = 2 * j + s;
          if (q1 != 0) u[j] = c_mul(u[j], twl[q1 * C::QC + C::LPC * ja]);
          Zc[(C::LPC * ja + j * C::QC) * C::P] = u[j];
        }
      }
      wave_sync();
      // forward pass B, pixel scaling, adjoint pass B^H: the same slots of this lane
#pragma unroll
      for (int jb = 0; jb < C::JB; ++jb) {
        const int j = sub + C::LPC * jb;
        const int q1 = 2 * j + s;
        float rr[C::QC];
        rload(cs, s, jb, rr);
        float2 v[C::QC];
#pragma unroll
        for (int k = 0; k < C::QC; ++k) v[k] = Zb[(C::LPC * jb * C::QC + k) * C::P];
        Dft<C::QC>::run(v);
#pragma unroll
        for (int q2 = 0; q2 < C::QC; ++q2) v[q2] = make_float2(v[q2].x * rr[q2], v[q2].y * rr[q2]);
        idft<C::QC>(v);
#pragma unroll
        for (int n2 = 0; n2 < C::QC; ++n2) {
          if (q1 != 0) v[n2] = c_mul_conj(v[n2], twb[(2 * C::LPC * jb + s) * C::QC + n2]);
          Zb[(C::LPC * jb * C::QC + n2) * C::P] = v[n2];
        }
      }
      wave_sync();
      // adjoint pass A^H, half-round s
#pragma unroll
      for (int ja = 0; ja < C::JA; ++ja) {
        float2 u[C::PH];
#pragma unroll
        for (int j = 0; j < C::PH; ++j) u[j] = Zc[(C::LPC * ja + j * C::QC) * C::P];
        idft<C::PH>(u);
        static_for<0, C::PH>([&](auto nc) {
          constexpr int n1 = decltype(nc)::value;
          const float2 t = (s == 0) ? u[n1] : rot<C::PC, -n1>(u[n1]);
          xacc[ja][n1] = c_add(xacc[ja][n1], t);
        });
      }
      wave_sync();
    });
#pragma unroll
    for (int ja = 0; ja < C::JA; ++ja)
#pragma unroll
      for (int n1 = 0; n1 < C::PH; ++n1) Zc[(C::LPC * ja + C::QC * n1) * C::P] = xacc[ja][n1];
    wave_sync();
  }
}

// Row stage adjoint: G'[iy][n'] = conj(w_N^{n' w}) sum_m Z'[iy][m] w_M^{-n' m}
// for n' < NZR, in place.
template <int N, int V>
__device__ __forceinline__ void row_stage_adjoint(float2* G, const float2* twr, const float2 (&fin)[FT<N, V>::PRNZ]) {
  using C = FT<N, V>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / C::RPW;
  const float2* twrb = twr + sub * C::QR;   // twrb[LPR jb QR + n2] = twr[q1 QR + n2]
#pragma unroll
  for (int rs = 0; rs < C::RSTEPS; ++rs) {
    const int row = stage_row(C::S, rs, wave, lane % C::RPW);
    if (C::RGUARD && row >= C::L) continue;
    float2* R = G + row * C::P;
    float2 y[C::JBR][C::QR];
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb)
#pragma unroll
      for (int q2 = 0; q2 < C::QR; ++q2) y[jb][q2] = R[sub + C::LPR * jb + C::PR * q2];
    wave_sync();
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb) {
      const int q1 = sub + C::LPR * jb;
      idft<C::QR>(y[jb]);
#pragma unroll
      for (int n2 = 0; n2 < C::QR; ++n2) {
        if (C::SX > 1 || q1 != 0) y[jb][n2] = c_mul_conj(y[jb][n2], twrb[C::LPR * jb * C::QR + n2]);
        R[q1 * C::QR + n2] = y[jb][n2];
      }
    }
    wave_sync();
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja) {
      float2 x[C::PR];
#pragma unroll
      for (int q1 = 0; q1 < C::PR; ++q1) x[q1] = R[sub + C::LPR * ja + q1 * C::QR];
      idft<C::PR>(x);
#pragma unroll
      for (int n1 = 0; n1 < C::PRNZ; ++n1) {
        float2 o = x[n1];
        if constexpr (C::SX > 1) o = c_mul_conj(o, fin[n1]);
        R[sub + C::LPR * ja + C::QR * n1] = o;
      }
    }
    wave_sync();
  }
}

// Row stage adjoint of column class W known at compile time (the adjoint of
// row_stage_w): the fold factor of output n' < NZR is conj(w_N^{QR n1 W}),
// applied as a constant rotation.
template <int N, int V, int W>
__device__ __forceinline__ void row_stage_adjoint_w(float2* G, const float2* twr) {
  using C = FT<N, V>;
  constexpr bool kFold = C::SX > 1 && W != 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane / C::RPW;
  const float2* twrb = twr + sub * C::QR;   // twrb[LPR jb QR + n2] = twr[q1 QR + n2]
#pragma unroll
  for (int rs = 0; rs < C::RSTEPS; ++rs) {
    const int row = stage_row(C::S, rs, wave, lane % C::RPW);
    if (C::RGUARD && row >= C::L) continue;
    float2* R = G + row * C::P;
    float2 y[C::JBR][C::QR];
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb)
#pragma unroll
      for (int q2 = 0; q2 < C::QR; ++q2) y[jb][q2] = R[sub + C::LPR * jb + C::PR * q2];
    wave_sync();
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb) {
      const int q1 = sub + C::LPR * jb;
      idft<C::QR>(y[jb]);
#pragma unroll
      for (int n2 = 0; n2 < C::QR; ++n2) {
        if (kFold || q1 != 0) y[jb][n2] = c_mul_conj(y[jb][n2], twrb[C::LPR * jb * C::QR + n2]);
        R[q1 * C::QR + n2] = y[jb][n2];
      }
    }
    wave_sync();
#pragma unroll
    for (int ja = 0; ja < C::JAR; ++ja) {
      float2 x[C::PR];
#pragma unroll
      for (int q1 = 0; q1 < C::PR; ++q1) x[q1] = R[sub + C::LPR * ja + q1 * C::QR];
      idft<C::PR>(x);
      static_for<0, C::PRNZ>([&](auto nc) {
        constexpr int n1 = decltype(nc)::value;
        float2 o = x[n1];
        if constexpr (kFold) o = rot<N / C::QR, -(n1 * W)>(o);
        R[sub + C::LPR * ja + C::QR * n1] = o;
      });
    }
    wave_sync();
  }
}

}  // namespace moff
