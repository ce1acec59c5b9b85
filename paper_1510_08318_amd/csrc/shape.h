// Tile shapes of the fused MOFF frame transform, shared by the host plan
// (which lays out the gather programs for them) and the HIP kernels.
//
// A workgroup of NT threads owns one channel, one residue class w of output
// columns (q = SX * m + w, m < M = N / SX) and a slice of time samples.  Per
// frame it gathers the folded aperture grid G[L][M] into LDS, transforms every
// row with an M-point DFT (PR x QR Stockham, in place, wave-owned rows), then
// every column with a pruned N-point DFT (PC x QC, L = (PC/2) QC nonzero
// inputs, two half-rounds in place, wave-owned columns), and accumulates |Y|^2
// in registers.
#pragma once

namespace moff {

struct FrameShape {
  int N = 0, NT = 0, SX = 0, PR = 0, QR = 0, PC = 0, QC = 0;
};

// Lanes per row of the row stage (RPW = 64 / row_lanes rows per wave and step).
constexpr int row_lanes(const FrameShape& S) { return S.QR < 4 ? S.QR : 4; }

// Row-stage ownership.  When one step of the row stage covers all L = N/2
// folded rows with more than one wave (NW * RPW == L), the rows are cut into
// 2 NW half-blocks of RPW/2 consecutive rows and wave w takes half-block w
// from the upper half of the grid and half-block NW + (w ^ 1) from the lower
// half, so that every wave's rows mix the aperture's sparse edges with its
// dense middle (the plan can then give each wave's lanes just its own rows
// to grid at little cost in balance).  The two half-blocks lie an odd number
// of half-blocks apart, so they start RPW/2 apart modulo RPW and a 16-lane
// group still touches 16 distinct banks.  Otherwise step rs of wave w takes
// rows (rs NW + w) RPW + r.  stage_row gives the row of step-row r < RPW.
constexpr bool paired_rows(const FrameShape& S) {
  return S.NT / 64 > 1 && (S.NT / 64) * (64 / row_lanes(S)) == S.N / 2;
}
constexpr int stage_row(const FrameShape& S, int rs, int wave, int r) {
  const int NW = S.NT / 64, RPW = 64 / row_lanes(S), H = RPW / 2;
  return paired_rows(S) ? (r < H ? wave * H + r : (NW + (wave ^ 1)) * H + (r - H)) : (rs * NW + wave) * RPW + r;
}

// LDS row pitch of the folded grid (complex elements) for M output columns per
// workgroup: odd, so that 16 lanes reading 16 different rows at the same column
// hit 16 different banks.
constexpr int grid_pitch(int M) { return M + 1; }

// Shape variants of the frame transform; the autotuner picks one per plan.
// Fields: {N, NT, SX, PR, QR, PC, QC}.  A variant with N == 0 does not exist.
constexpr int kMaxVariants = 2;

constexpr FrameShape frame_shape(int N, int V = 0) {
  return N == 8   ? (V == 0 ? FrameShape{8, 64, 1, 4, 2, 4, 2} : FrameShape{})
       : N == 16  ? (V == 0 ? FrameShape{16, 64, 1, 4, 4, 4, 4} : FrameShape{})
       : N == 32  ? (V == 0 ? FrameShape{32, 64, 1, 8, 4, 8, 4} : FrameShape{})
       : N == 64  ? (V == 0 ? FrameShape{64, 128, 1, 8, 8, 8, 8} : FrameShape{})
       : N == 128 ? (V == 0 ? FrameShape{128, 256, 2, 8, 8, 16, 8} : FrameShape{128, 256, 1, 16, 8, 16, 8})
       : N == 256 ? (V == 0 ? FrameShape{256, 256, 4, 8, 8, 16, 16} : FrameShape{256, 512, 2, 16, 8, 16, 16})
                  : FrameShape{};
}

// Waves per workgroup of the reduced-precision (matrix-core) frame transform:
// matrix waves run the two transform stages, gather waves ingest and grid.
constexpr int mfma_waves(int N) { return N == 128 ? 8 : 2; }
constexpr int mfma_gather_waves(int N) { return N == 128 ? 4 : 2; }

// Dynamic LDS one workgroup may take: a compute unit's 160 KB less room for
// the kernels' static arrays (the launch rejects anything larger).
constexpr int kMfmaLdsMax = 159 * 1024;

// Dynamic-LDS layout of the reduced-precision kernel, byte offsets.  The two
// buffers of calibrated samples e[n_ant + 1] (last slot zero) and the kernel
// taps come first so that gather entries can address them with 16-bit byte
// offsets; the two 16-bit grids Eg [N/2][pitch] and the two transposed
// row-stage outputs Zt [N][pitch] follow, then per-antenna gains and types,
// the row stage's phase-factor operands (read from LDS one step at a time),
// then (optionally) the program.  Gather entries address buffer 0; buffer 1
// of each pair lies one *_stride further on.
struct MfmaLayout {
  int pitch;   // 16-bit elements per Eg / Zt row
  int e, e_stride, k, eg, eg_stride, zt, zt_stride, gl, ty, wt, prog;
};

constexpr int align_up(int x, int a) { return (x + a - 1) / a * a; }

constexpr MfmaLayout mfma_layout(int N, int n_taps, int n_ant) {
  const int L = N / 2, pitch = 2 * L + 8;
  MfmaLayout m{};
  m.pitch = pitch;
  m.e = 0;
  m.e_stride = 8 * (n_ant + 1);
  m.k = 2 * m.e_stride;
  m.eg = align_up(m.k + 8 * n_taps, 16);
  m.eg_stride = 2 * L * pitch;
  m.zt = m.eg + 2 * m.eg_stride;
  m.zt_stride = 2 * N * pitch;
  m.gl = m.zt + 2 * m.zt_stride;
  m.ty = m.gl + 8 * n_ant;
  // the row stage's phase-factor operands, [N/64][2][N/64][2][64] x 16 bytes
  m.wt = align_up(m.ty + 4 * n_ant, 16);
  m.prog = m.wt + (L / 32) * 2 * (L / 32) * 2 * 64 * 16;
  return m;
}

}  // namespace moff
