// Host tables of the visibility-route (FX) image (fx.hip), built on first use
// by fx_tables.cpp.  Pure C++17, no HIP.
#pragma once

#include <cstdint>
#include <vector>

#include "plan.h"

namespace moff {

// Tables of the visibility-route image (Sec. 2, eq. dirty-image-FX with
// eq. e-field-conv), built on first use:
//   ptr / ab : CSR over (type pair p * n_types + q, footprint offset cell
//              (iy0_a - iy0_b + L - 1) * NL + ix0_a - ix0_b + L - 1) of the
//              ordered antenna pairs (a of type p, b of type q), in ascending
//              (a, b) order; a == b only when the zero-spacing terms are kept.
//              Only rows at or before their mirror row (types swapped, offset
//              negated), which holds the conjugate sum, have entries.  An entry
//              is min(a, b) * n_ant + max(a, b), the upper-triangle visibility,
//              with kFxConjBit set when a > b (read it conjugated).
//   xcorr    : per type pair, X[u][v] = sum K_p[s][t] conj(K_q[s - u + k_q - 1][t - v + k_q - 1])
//              on a (k_p + k_q - 1)^2 support, stored [pair][xs][xs] as float32 (re, im).
constexpr uint32_t kFxConjBit = 0x80000000u;

struct FxTables {
  int NL = 0, xs = 0;
  std::vector<int32_t> ptr, ab;
  std::vector<float> xcorr;
};
void build_fx_tables(const HostPlan& hp, bool keep_autos, FxTables* t);

}  // namespace moff
