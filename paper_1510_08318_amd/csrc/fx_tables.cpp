// Host tables of the visibility-route (FX) image (declared in fx_tables.h).
// Pure C++17, no HIP.
#include "fx_tables.h"

#include <algorithm>
#include <complex>

namespace moff {

void build_fx_tables(const HostPlan& hp, bool keep_autos, FxTables* t) {
  const int na = hp.n_ant, L = hp.L, NL = 2 * L - 1, nt = hp.n_ktypes;
  int kmax = 1;
  for (int p = 0; p < nt; ++p) kmax = std::max(kmax, static_cast<int>(hp.ktype_k[p]));
  t->NL = NL;
  t->xs = 2 * kmax - 1;
  // pair responses: cross-correlation of two tables placed at the same cell
  const int xs = t->xs;
  t->xcorr.assign(static_cast<size_t>(nt) * nt * xs * xs * 2, 0.f);
  for (int p = 0; p < nt; ++p)
    for (int q = 0; q < nt; ++q) {
      const int ka = hp.ktype_k[p], kb = hp.ktype_k[q], side = ka + kb - 1;
      const float* Ka = hp.kvals.data() + 2 * static_cast<size_t>(hp.ktype_off[p]);
      const float* Kb = hp.kvals.data() + 2 * static_cast<size_t>(hp.ktype_off[q]);
      std::vector<std::complex<double>> X(static_cast<size_t>(side) * side);
      for (int s0 = 0; s0 < ka; ++s0)
        for (int s1 = 0; s1 < ka; ++s1) {
          const std::complex<double> x(Ka[2 * (s0 * ka + s1)], Ka[2 * (s0 * ka + s1) + 1]);
          for (int r0 = 0; r0 < kb; ++r0)
            for (int r1 = 0; r1 < kb; ++r1) {
              const std::complex<double> y(Kb[2 * (r0 * kb + r1)], -Kb[2 * (r0 * kb + r1) + 1]);
              X[static_cast<size_t>(s0 - r0 + kb - 1) * side + (s1 - r1 + kb - 1)] += x * y;
            }
        }
      float* dst = t->xcorr.data() + static_cast<size_t>(p * nt + q) * xs * xs * 2;
      for (int u = 0; u < side; ++u)
        for (int v = 0; v < side; ++v) {
          dst[2 * (u * xs + v)] = static_cast<float>(X[static_cast<size_t>(u) * side + v].real());
          dst[2 * (u * xs + v) + 1] = static_cast<float>(X[static_cast<size_t>(u) * side + v].imag());
        }
    }
  // CSR of the ordered pairs by (type pair, offset cell), by counting sort.
  // The pair (b, a) lands in the mirror row -- types swapped, offset negated --
  // with the conjugate visibility, so only rows that do not follow their mirror
  // hold entries; the device sums those and writes each mirror as the
  // conjugate.  An entry names the upper-triangle element min(a, b) n_ant +
  // max(a, b), with the top bit set when a > b (conjugate on reading).
  const size_t rows = static_cast<size_t>(nt) * nt * NL * NL;
  auto row_of = [&](int a, int b) {
    const int tp = hp.ant_ktype[a] * nt + hp.ant_ktype[b];
    const int dy = hp.iy0[a] - hp.iy0[b] + L - 1, dx = hp.ix0[a] - hp.ix0[b] + L - 1;
    return (static_cast<size_t>(tp) * NL + dy) * NL + dx;
  };
  auto canonical = [&](int a, int b) { return row_of(a, b) <= row_of(b, a); };
  auto keep = [&](int a, int b) { return (a != b || keep_autos) && canonical(a, b); };
  t->ptr.assign(rows + 1, 0);
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < na; ++b)
      if (keep(a, b)) ++t->ptr[row_of(a, b) + 1];
  for (size_t r = 0; r < rows; ++r) t->ptr[r + 1] += t->ptr[r];
  t->ab.assign(static_cast<size_t>(t->ptr[rows]), 0);
  std::vector<int32_t> fill(t->ptr.begin(), t->ptr.end() - 1);
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < na; ++b)
      if (keep(a, b)) {
        const uint32_t upper = static_cast<uint32_t>(std::min(a, b)) * na + std::max(a, b);
        t->ab[static_cast<size_t>(fill[row_of(a, b)]++)] = static_cast<int32_t>(upper | (a > b ? kFxConjBit : 0u));
      }
}

}  // namespace moff
