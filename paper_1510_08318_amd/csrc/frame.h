// The per-frame transform of the fused and staged kernels: the zero-padded
// 2-D DFT of one channel-frame, restricted to the output columns
// q = SX * m + w of one workgroup, staged in LDS (Sec. 3, spatial Fourier
// transform; zero padding to twice the aperture per axis, Sec. 6.1).
//
// Layout in LDS: the folded aperture grid G[iy][n'] (iy < L, n' < M, row pitch
// ZP complex elements), where
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

template <int N_>
struct FT {
  static constexpr FrameShape S = frame_shape(N_);
  static constexpr int N = N_, NT = S.NT, SX = S.SX, M = N / SX, L = N / 2, NW = NT / 64;
  static constexpr int PR = S.PR, QR = S.QR, PC = S.PC, QC = S.QC, LPC = S.LPC;
  static constexpr int NZR = L < M ? L : M;
  static constexpr int PRNZ = NZR / QR;          // nonzero inputs of the row pass A
  static constexpr int JBR = PR / QR;            // row pass-B jobs per lane
  static constexpr int RPW = 64 / QR;            // rows per wave per step
  static constexpr int RSTEPS = (L + NW * RPW - 1) / (NW * RPW);
  static constexpr bool RGUARD = (L % (NW * RPW)) != 0;
  static constexpr int PH = PC / 2;              // column pass-A length per half-round
  static constexpr int JA = QC / LPC;            // column pass-A jobs per lane
  static constexpr int JB = PH / LPC;            // column pass-B jobs per lane per half-round
  static constexpr int CPW = 64 / LPC;           // columns per wave per step
  static constexpr int CSTEPS = (M + NW * CPW - 1) / (NW * CPW);
  static constexpr bool CGUARD = (M % (NW * CPW)) != 0;
  static constexpr int ZP = grid_pitch(M);
  static constexpr int NACC = CSTEPS * 2 * JB * QC;
  static_assert(PR * QR == M && PC * QC == N, "bad factorisation");
  static_assert(PH * QC == L, "column half-round must fill the L slots");
  static_assert(QC % LPC == 0 && PH % LPC == 0 && 64 % LPC == 0 && 64 % QR == 0 && PR % QR == 0, "bad lanes");
  static_assert(NZR % QR == 0, "row pruning must align with the decimation");
};

// Row stage: Z[iy][m] = sum_{n'} G[iy][n'] w_N^{n' w} w_M^{n' m}, in place.
// tw: LDS twiddles w_N^k, k < N.
template <int N>
__device__ __forceinline__ void row_stage(float2* G, const float2* tw, int w) {
  using C = FT<N>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n2 = lane % C::QR;
#pragma unroll
  for (int rs = 0; rs < C::RSTEPS; ++rs) {
    const int row = (rs * C::NW + wave) * C::RPW + lane / C::QR;
    if (C::RGUARD && row >= C::L) continue;
    float2* R = G + row * C::ZP;
    float2 x[C::PR];
#pragma unroll
    for (int n1 = 0; n1 < C::PRNZ; ++n1) {
      x[n1] = R[C::QR * n1 + n2];
      if constexpr (C::SX > 1) x[n1] = c_mul(x[n1], tw[((C::QR * n1 + n2) * w) & (N - 1)]);
    }
    dft_pruned<C::PR, C::PRNZ>(x);
#pragma unroll
    for (int q1 = 1; q1 < C::PR; ++q1) x[q1] = c_mul(x[q1], tw[(C::SX * n2 * q1) & (N - 1)]);
    wave_sync();
#pragma unroll
    for (int q1 = 0; q1 < C::PR; ++q1) R[q1 * C::QR + n2] = x[q1];
    wave_sync();
    float2 y[C::JBR][C::QR];
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb) {
      const int q1 = n2 + C::QR * jb;
#pragma unroll
      for (int k = 0; k < C::QR; ++k) y[jb][k] = R[q1 * C::QR + k];
    }
    wave_sync();
#pragma unroll
    for (int jb = 0; jb < C::JBR; ++jb) {
      const int q1 = n2 + C::QR * jb;
      Dft<C::QR>::run(y[jb]);
#pragma unroll
      for (int q2 = 0; q2 < C::QR; ++q2) R[q1 + C::PR * q2] = y[jb][q2];
    }
    wave_sync();
  }
}

// Column stage: Y[r][m] = sum_{iy < L} Z[iy][m] w_N^{iy r} for r < N, in place,
// handing every output to sink(acc_index, r, m, value) with a compile-time
// acc_index in [0, NACC).
template <int N, class Sink>
__device__ __forceinline__ void col_stage(float2* G, const float2* tw, Sink&& sink) {
  using C = FT<N>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane % C::LPC;
#pragma unroll
  for (int cs = 0; cs < C::CSTEPS; ++cs) {
    const int col = (cs * C::NW + wave) * C::CPW + lane / C::LPC;
    if (C::CGUARD && col >= C::M) continue;
    float2* Zc = G + col;
    float2 z[C::JA][C::PH];
#pragma unroll
    for (int ja = 0; ja < C::JA; ++ja) {
      const int n2 = lc + C::LPC * ja;
#pragma unroll
      for (int n1 = 0; n1 < C::PH; ++n1) z[ja][n1] = Zc[(C::QC * n1 + n2) * C::ZP];
    }
    wave_sync();
    static_for<0, 2>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
#pragma unroll
      for (int ja = 0; ja < C::JA; ++ja) {
        const int n2 = lc + C::LPC * ja;
        float2 u[C::PH];
        static_for<0, C::PH>([&](auto nc) {
          constexpr int n1 = decltype(nc)::value;
          u[n1] = s ? rot<C::PC, n1>(z[ja][n1]) : z[ja][n1];
        });
        Dft<C::PH>::run(u);
#pragma unroll
        for (int j = 0; j < C::PH; ++j) {
          const int q1 = 2 * j + s;
          if (q1 != 0) u[j] = c_mul(u[j], tw[(n2 * q1) & (N - 1)]);
          Zc[(j * C::QC + n2) * C::ZP] = u[j];
        }
      }
      wave_sync();
      float2 v[C::JB][C::QC];
#pragma unroll
      for (int jb = 0; jb < C::JB; ++jb) {
        const int j = lc + C::LPC * jb;
#pragma unroll
        for (int k = 0; k < C::QC; ++k) v[jb][k] = Zc[(j * C::QC + k) * C::ZP];
      }
      wave_sync();
#pragma unroll
      for (int jb = 0; jb < C::JB; ++jb) {
        const int j = lc + C::LPC * jb;
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

// Output pixel coordinates (r, m) of accumulator `idx` for this lane; the
// same mapping col_stage hands to its sink.
template <int N>
__device__ __forceinline__ void acc_pixel(int idx, int& r, int& col) {
  using C = FT<N>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q2 = idx % C::QC;
  const int jb = (idx / C::QC) % C::JB;
  const int s = (idx / (C::QC * C::JB)) % 2;
  const int cs = idx / (C::QC * C::JB * 2);
  const int j = lane % C::LPC + C::LPC * jb;
  col = (cs * C::NW + wave) * C::CPW + lane / C::LPC;
  r = 2 * j + s + C::PC * q2;
}

}  // namespace moff
