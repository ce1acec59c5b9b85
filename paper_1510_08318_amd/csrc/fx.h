// Visibility-route (FX) image on the device: launch arguments of fx.hip (its
// host tables are built by fx_tables.cpp, declared in fx_tables.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace moff {

// Visibility-route (FX) image of one integration, for cross-checks of the MOFF
// image on the device (fx.hip).  NL = 2L - 1 lags per axis, NTP = n_types^2
// ordered pairs of table types.
struct FxArgs {
  const void* E;
  const float2* gains;         // [n_chan][n_ant] or null (unit gains)
  int n_ant, n_chan, n_types;  // n_chan: channels of E, gains and out
  int c0, n_launch;            // this launch's channels c0 .. c0 + n_launch - 1 (workspace holds n_launch)
  int64_t n_time;
  int N, L, NL, xs;            // xs: side of each pair-response table
  const int* pair_ptr;         // [NTP * NL * NL + 1] CSR over (type pair, footprint offset)
  const int* pair_ab;          // [entries] upper-triangle index of V, kFxConjBit: read conjugated
  const int* ktype_k;          // [n_types]
  const float2* xcorr;         // [NTP][xs][xs] pair responses of the tables
  const float2* tw;            // [N] exp(+2 pi i k / N)
  float2* V;                   // [n_launch][n_ant][n_ant] workspace (upper triangle used)
  float2* H;                   // [n_launch][NTP][NL][NL] workspace
  float2* R;                   // [n_launch][NL][NL] workspace
  float2* Z;                   // [n_launch][NL][N] workspace
  float* out;                  // [n_chan][N][N]
  double scale;
};
hipError_t launch_fx(const FxArgs& a, bool ci4, hipStream_t st);
}  // namespace moff
