// Kernel argument blocks and launchers (host-callable), shared by kernels.hip
// and the C ABI.  Pointers are device pointers unless stated.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace moff {

enum { kModePartial = 0, kModeAccum = 1, kModeFinal = 2 };

// XCDs of the device: workgroups are dispatched to them round-robin by index,
// so workgroups whose indices agree modulo kXcds share one L2.
constexpr int kXcds = 8;

struct FusedArgs {
  const void* E;               // [T][C][n_ant] c64 or ci4
  const float2* gains;         // [C][n_ant] or nullptr
  const uint4* prog;           // [SX][prog_len / 4][NT] (HostPlan::Variant::prog4)
  const float4* progw;         // entry weights laid out like prog (HostPlan::Variant::progw) or nullptr
  const int* cell0;            // [SX][NT] first folded cell of each lane
  int prog_len;
  int wave_rows;               // each wave grids only the rows it transforms (HostPlan::Variant::wave_rows)
  int dst_entries;             // program entries carry their cell (HostPlan::Variant::dst_entries)
  int progress_prio;           // issue priority by slice progress (several workgroups per CU)
  const float2* weights;       // [SX][n_weights]
  int n_weights;
  const float2* tw;            // [N]
  const int* ant_type;         // [n_ant]
  int n_ant, n_chan, n_types;
  int64_t n_time;
  int slices;
  float* out;                  // partial: [slices][C][N][N]; accum: S [C][N][N]; final: image
  double* outA;                // partial: [slices][C][types]; accum: A [C][types]
  const double* Pp;            // [types][N][N]
  double scale;
  int subtract;
  int mode;                    // kModePartial / kModeAccum / kModeFinal
  // Blocked accumulation: a workgroup whose slice holds more than kBlockFrames
  // samples adds its float32 register sums into float64 running sums every
  // kBlockFrames samples (acc64: N^2 doubles per (column class, channel,
  // slice) work item, private to the item's workgroup).  Null when no slice
  // is that long.
  double* acc64;
};

// Samples summed in float32 registers before they are added to a float64
// running sum.  The float32 part then contributes at most (kBlockFrames - 1)
// units of rounding (2^-24 each) relative to the accumulated power of a pixel
// in the worst case, and about sqrt(kBlockFrames) / 3 units for roundings of
// random sign; the float64 running sums keep that from growing with the
// length of the integration.  A block of 256 covers the HERA-shaped and
// calibration integrations (256 and 128 samples) in one slice without a
// running-sum round trip through memory.
constexpr int kBlockFrames = 256;

struct ReduceArgs {
  const float* S_part;
  const double* A_part;
  const double* Pp;
  float* out;
  double* outA;
  int N, n_chan, n_types, slices;
  int final_image, subtract;
  double scale;
};

struct GridArgs {
  const void* E;
  const float2* gains;
  const float2* ktab;          // [n_taps]
  const int* csr_ptr;          // [L*L + 1]
  const int* csr_ant;
  const int* csr_tap;
  const int* ant_type;
  float2* Eg;                  // [T][C][L][L]
  double* A;                   // [C][types]
  int n_ant, n_chan, n_taps, n_types, L;
  int64_t n_time;
};

struct Fft2Args {
  const float2* Eg;            // [F][L][L]
  float2* Y;                   // [F][N][N]
  const float2* tw;            // [N]
};

struct DetectArgs {
  const float2* Y;             // [T][C][N][N]
  float* S;                    // [C][N][N]
  int N, n_chan;
  int64_t n_time;
};

struct FinalizeArgs {
  const float* S;
  const double* A;
  const double* Pp;
  float* out;
  int N, n_chan, n_types, subtract;
  double scale;
};

// Gain-gradient (adjoint) kernels.
struct AdjFftArgs {
  const float2* Y;             // [F][N][N] image fields of a time chunk, frame f = t * n_chan + c
  const float* R;              // [C][N][N] dL/dI
  float2* Gp;                  // [F][SX][L][NZR] folded adjoint grids
  const float2* tw;            // [N]
  int n_chan;
};

struct DegridArgs {
  const void* E;               // [T_chunk][C][n_ant] raw samples of the chunk
  const float2* Gp;            // [T_chunk * C][SX][L][NZR]
  const float2* weights;       // [SX][NJ * n_taps] (variant 0)
  const int* ant_type;
  const int* ant_cells;        // [n_ant][2] = (ix0, iy0)
  const int* ktype_k;          // [types]
  const int* ktype_off;        // [types] first tap of each type
  double2* D;                  // [C][n_ant] += sum_t conj(E) d
  double* Q;                   // [C][n_ant] += sum_t |E|^2
  int n_ant, n_chan, n_taps, SX, L, M, NZR, NJ;
  int64_t n_time;
};

struct GradFinalArgs {
  const double2* D;
  const double* Q;
  const float* R;              // [C][N][N]
  const double* Pp;            // [types][N][N]
  const float2* gains;         // [C][n_ant] or nullptr
  const int* ant_type;
  float2* grad;                // [C][n_ant]
  int N, n_ant, n_chan, n_types, subtract;
  double scale;                // 2 s / T
};

// Reduced-precision fused kernel (MOFF_MFMA_*): one workgroup per (channel,
// time slice); same epilogue modes and outputs as FusedArgs.
struct MfmaArgs {
  const void* E;               // [T][C][n_ant] c64 or ci4
  const float2* gains;         // [C][n_ant] or nullptr
  const GatherEntry* prog;     // [prog_len][gather lanes]
  int prog_len;
  int prog_in_lds;             // copy the program into LDS (mfma_prog_in_lds)
  const float2* ktab;          // [n_taps] kernel taps, all types back to back
  int n_taps;
  const uint16_t* dft;         // phase-factor operands (HostPlan::Mfma::dft), 16-byte aligned
  const int* ant_type;
  int n_ant, n_chan, n_types;
  int64_t n_time;
  int slices;
  float* out;
  double* outA;
  const double* Pp;
  double scale;
  int subtract;
  int mode;
};

size_t mfma_lds_bytes(int N, int n_taps, int n_ant, int prog_len, bool prog_in_lds);
bool mfma_prog_in_lds(int N, int n_taps, int n_ant, int prog_len);
int mfma_threads(int N);
hipError_t launch_mfma(const MfmaArgs& a, int N, int prec, bool ci4, int grid, hipStream_t st);
int mfma_blocks_per_cu(int N, int prec, bool ci4, size_t lds);

// uv-plane autocorrelation removal (uv_autocorr.hip): `S` is the per-channel
// input (accumulated squared image, or dL/dI for the adjoint shift), `out` the
// per-channel output, both [C][N][N]; Pn = sum_p n_p P_p and a0 = sum_p n_p sum|K_p|^2.
struct UvArgs {
  const float* S;
  const double* Pn;            // [N][N]
  float* out;
  int N, n_chan;
  double a0, scale;
};
hipError_t launch_uv_finalize(const UvArgs& a, hipStream_t st);
hipError_t launch_uv_adjoint_shift(const UvArgs& a, hipStream_t st);

// Fused gain adjoint: one workgroup per (column class, channel, time slice) runs
// ingest, gridding, the frame transform, the pixel-wise product with R, the
// adjoint transform and the degridding for every frame, and writes per-antenna
// partial sums Dp[(slice * SX + w)][C][n_ant] += conj(E) d over its frames.
struct AdjFusedArgs {
  const void* E;               // [T][C][n_ant] c64 or ci4
  const float2* gains;         // [C][n_ant] or nullptr
  const uint4* prog;           // [SX][prog_len / 4][NT] (the forward gather program)
  const float4* progw;         // its entry weights, or nullptr
  const int* cell0;            // [SX][NT]
  int prog_len;
  int wave_rows;               // as FusedArgs::wave_rows
  int dst_entries;             // as FusedArgs::dst_entries
  int progress_prio;           // as FusedArgs::progress_prio
  const float2* weights;       // [SX][n_weights]
  int n_weights;
  const float2* tw;            // [N]
  const uint32_t* slots;       // [NT][kAdjSlots][2] (HostPlan::Variant::slots)
  const float* Rl;             // [C][SX][NACC * NT] dL/dI per lane (launch_adjoint_sensitivity)
  int n_ant, n_chan, n_taps;
  int64_t n_time;
  int slices;
  double2* Dp;                 // [slices * SX][C][n_ant]
};
// wps: waves per SIMD the adjoint's registers are sized for, 1 .. adjoint_waves_max(N)
int adjoint_waves_max(int N);
hipError_t launch_adjoint_fused(const AdjFusedArgs& a, int N, int V, bool ci4, int wps, int grid, hipStream_t st);
int adjoint_fused_blocks_per_cu(int N, int V, bool ci4, int wps, size_t lds);
// Values one channel's workgroups of shape variant V hold per lane, summed
// over the lanes and output classes: SX * NACC * NT (at least N^2; more where
// some lanes of a small grid own no column).  The size, per channel and time
// slice, of the blocked-accumulation running sums and of Rl.
size_t fused_lane_values(int N, int V);
// Rl [C][fused_lane_values(N, V)] for shape variant V from R [C][N][N].
hipError_t launch_adjoint_sensitivity(const float* R, int N, int V, int n_chan, float* Rl, hipStream_t st);
// Q[c][a] = sum_t |E[t][c][a]|^2 (float64); D[c][a] = sum_k Dp[k][c][a] over `parts` partials.
hipError_t launch_antenna_power(const void* E, bool ci4, int64_t n_time, int n_chan, int n_ant, double* Q,
                                hipStream_t st);
hipError_t launch_adjoint_reduce(const double2* Dp, int parts, int n_chan, int n_ant, double2* D, hipStream_t st);

hipError_t launch_adjoint_fft2(const AdjFftArgs& a, int N, int64_t n_frames, hipStream_t st);
hipError_t launch_degrid(const DegridArgs& a, bool ci4, hipStream_t st);
hipError_t launch_grad_final(const GradFinalArgs& a, hipStream_t st);

// Fused kernel of grid size N, shape variant V (shape.h), one work item
// (column class, channel, time slice) per workgroup of a `grid`-sized launch.
size_t fused_lds_bytes(int N, int V, int n_weights, int n_ant);
hipError_t launch_fused(const FusedArgs& a, int N, int V, bool ci4, int grid, hipStream_t st);
int fused_blocks_per_cu(int N, int V, bool ci4, size_t lds);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_grid(const GridArgs& a, bool ci4, hipStream_t st);
hipError_t launch_self_power(const GridArgs& a, bool ci4, hipStream_t st);
hipError_t launch_fft2(const Fft2Args& a, int N, int64_t n_frames, hipStream_t st);
hipError_t launch_detect(const DetectArgs& a, hipStream_t st);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);  // bytes: multiple of 4

}  // namespace moff
