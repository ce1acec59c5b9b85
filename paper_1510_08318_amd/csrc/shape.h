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
  int N, NT, SX, PR, QR, PC, QC;
};

// LDS row pitch of the folded grid (complex elements) for M output columns per
// workgroup: odd, so that 16 lanes reading 16 different rows at the same column
// hit 16 different banks.
constexpr int grid_pitch(int M) { return M + 1; }

constexpr FrameShape frame_shape(int N) {
  return N == 8   ? FrameShape{8, 64, 1, 4, 2, 4, 2}
       : N == 16  ? FrameShape{16, 64, 1, 4, 4, 4, 4}
       : N == 32  ? FrameShape{32, 64, 1, 8, 4, 8, 4}
       : N == 64  ? FrameShape{64, 128, 1, 8, 8, 8, 8}
       : N == 128 ? FrameShape{128, 256, 2, 8, 8, 16, 8}
       : N == 256 ? FrameShape{256, 256, 4, 8, 8, 16, 16}
                  : FrameShape{0, 0, 0, 0, 0, 0, 0};
}

}  // namespace moff
