// Host side of a MOFF plan: everything computed once per geometry
// (Sec. 3: the antenna-to-grid mapping and W(r) need only be determined once).
// Pure C++17, no HIP; compiled without FP contraction so that the footprint
// cell of every antenna is decided by the same IEEE double operations as in
// its definition.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/moff.h"
#include "shape.h"

namespace moff {

// A gather entry of the fused kernel: 8 bytes, read coalesced by lane.
//   x bits  0..11 : antenna slot in LDS (n_ant = the all-zero slot)
//   x bits 12..22 : weight index into the workgroup's complex weight table
//   x bit  31     : last entry of its cell -> store the running sum
//   y             : LDS element iy * ZP + n' of the folded-grid cell (if stored)
// The device form keeps the x words only (HostPlan::Variant::prog4), or with
// destination-carrying entries (Variant::dst_entries) slot | element << 12 |
// first-entry-of-its-cell << 30.
struct GatherEntry {
  uint32_t x, y;
};

constexpr uint32_t kStoreBit = 0x80000000u;
constexpr uint32_t kFirstBit = 0x40000000u;

// Antenna slots of the fused adjoint: each lane degrids up to kAdjSlots whole
// antennas, two words per slot:
//   w0 bits 0..11 antenna (kAdjEmpty = none), bits 12..23 first tap of its
//      table, bits 24..27 table side k;   w1 = ix0 | iy0 << 16.
constexpr int kAdjSlots = 4;
constexpr uint32_t kAdjEmpty = 0xFFFu;
constexpr int kMaxAnt = 4000;
constexpr int kMaxTypes = 4;
constexpr int kMaxK = 15;

struct HostPlan {
  // geometry (copied)
  int n_ant = 0, n_ktypes = 0, n_chan = 0, N = 0, L = 0;
  uint32_t flags = 0;
  double cell_m = 0;
  std::vector<double> ant_xy, freq_hz, lm_per_pixel;
  std::vector<int32_t> ktype_k, ktype_off, ant_ktype;
  std::vector<float> kvals;                 // float32 (re, im) as given, all types back to back
  int n_taps = 0;                            // total table entries over all types

  // placement
  std::vector<int32_t> ix0, iy0;

  // staged gridding: CSR over the L x L aperture cells, entries sorted by antenna
  std::vector<int32_t> csr_ptr;              // [L*L + 1]
  std::vector<int32_t> csr_ant, csr_tap;     // [nnz]

  // power patterns, float64 [n_ktypes][N][N] in image pixel order
  std::vector<double> Pp;
  // uv-plane autocorrelation rule: Pn = sum_p n_p P_p [N][N] and
  // a0 = sum_p n_p sum |K_p|^2 (the tables' autocorrelation at zero lag)
  std::vector<double> Pn;
  double a0 = 0.0;

  // twiddles w_N^k = exp(+2 pi i k / N), k < N, float32 (re, im)
  std::vector<float> twiddle;

  // fused frame transform, one entry per shape variant (see shape.h)
  struct Variant {
    FrameShape shape{};
    int M = 0, NZR = 0, NJ = 0, ZP = 0;       // ZP: LDS row pitch of the folded grid
    int prog_len = 0;                        // entries per lane (padded to a multiple of 4)
    std::vector<GatherEntry> prog;           // [SX][prog_len][NT], host form with each store's LDS cell
    // Device form: the x words only, four consecutive entries of a lane side by
    // side, [SX][prog_len / 4][NT][4]; a lane's stores fill consecutive folded
    // cells (iy, n') in row-major order from its first cell cell0[w][lane].
    std::vector<uint32_t> prog4;
    std::vector<int32_t> cell0;              // [SX][NT]
    // When every weight of every class is real (real tables, no fold factor),
    // progw holds each entry's weight, laid out like prog4, so the kernel
    // reads it with the entry instead of looking it up in LDS; else empty.
    std::vector<float> progw;
    // Every wave's lanes grid exactly the folded rows that wave transforms in
    // the row stage (one block of 64 / row_lanes rows per wave), so no
    // workgroup barrier is needed between the two.
    bool wave_rows = false;
    // Device-form entries carry their cell's LDS element (see GatherEntry).
    bool dst_entries = false;
    std::vector<float> weights;              // [SX][NJ * n_taps] complex: K[tap] * w_SX^(j w)
    int n_weights() const { return NJ * n_taps_; }
    int n_taps_ = 0;
    std::vector<uint32_t> slots;             // [NT][kAdjSlots][2]; empty if the antennas do not fit
  };
  std::vector<Variant> variants;
  int max_cell_entries = 0;

  // reduced-precision frame transform (MOFF_MFMA_*): dense DFT matrices on the
  // matrix cores; see mfma.hip for the operand layout
  struct Mfma {
    int prec = 0;                            // 0: off, 1: binary16, 2: bfloat16
    int NT = 0, pitch = 0, prog_len = 0, grid_base = 0;
    std::vector<GatherEntry> prog;           // [prog_len][NT]; LDS byte offsets (mfma_layout)
    std::vector<uint16_t> dft;               // [2][N/64][2][N/64][2][64][8] operand bit patterns
  } mfma;
};

// 16-bit encodings of a float64 value, rounded to nearest (ties to even).
uint16_t to_binary16(double x);
uint16_t to_bfloat16(double x);

// Validate the geometry and build every host table.  Returns MOFF_OK or the
// status describing the first problem; `why` gets a human-readable reason.
moff_status build_host_plan(const moff_geometry* g, HostPlan* hp, std::string* why);

}  // namespace moff
