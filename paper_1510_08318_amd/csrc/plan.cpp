// Host plan construction (see plan.h).  Built with -ffp-contract=off.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace moff {

namespace {

constexpr double kC = 299792458.0;  // speed of light, m/s
constexpr double kTwoPi = 6.283185307179586476925286766559;

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// exp(+2 pi i num / den) with exact values on the quarter turns.
std::complex<double> unit_root(long long num, long long den) {
  long long r = ((num % den) + den) % den;
  if ((4 * r) % den == 0) {
    switch ((4 * r) / den) {
      case 0: return {1.0, 0.0};
      case 1: return {0.0, 1.0};
      case 2: return {-1.0, 0.0};
      default: return {0.0, -1.0};
    }
  }
  double ang = kTwoPi * static_cast<double>(r) / static_cast<double>(den);
  return {std::cos(ang), std::sin(ang)};
}

moff_status fail(std::string* why, moff_status s, const char* msg) {
  if (why) *why = msg;
  return s;
}

// Round |x| to `sig` significant bits (ties to even) with the quantum never
// below 2^min_q (gradual underflow); exact in float64 because the scalings are
// powers of two.
double round_sig(double ax, int sig, int min_q) {
  if (ax == 0.0) return 0.0;
  int e = 0;
  (void)std::frexp(ax, &e);                 // ax = m 2^e, 0.5 <= m < 1
  const int q = std::max(e - sig, min_q);   // quantum 2^q
  return std::nearbyint(std::ldexp(ax, -q)) * std::ldexp(1.0, q);
}

// Contiguous greedy split of `cost` (in order) over at most `lanes` lanes with
// the smallest per-lane maximum; returns that maximum.
long long balanced_split(const std::vector<int>& cost, int lanes) {
  auto lanes_needed = [&](long long B) {
    int n = 1;
    long long cur = 0;
    for (int c : cost) {
      if (cur + c > B) {
        ++n;
        cur = 0;
      }
      cur += c;
    }
    return n;
  };
  long long lo = 1, hi = 1;
  for (int c : cost) {
    lo = std::max<long long>(lo, c);
    hi += c;
  }
  while (lo < hi) {
    long long mid = (lo + hi) / 2;
    if (lanes_needed(mid) <= lanes) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Tables of the reduced-precision (matrix-core) path.  The gather program is
// the cell-keyed CSR split into balanced per-lane slices for the gather waves,
// encoded in LDS byte offsets.  The phase-factor operands are those of the
// base half of each transform: the row stage's output columns q < N/2 and the
// column stage's output rows r < N/2, whose partners N - q and N - r follow by
// conjugation.  Index 0 carries the two real self-conjugate phase vectors
// (q - N/2 = -N/2 and 0) as real and imaginary part of one slot.  Values are
// correctly rounded from float64 to binary16 or bfloat16, laid out in the
// register order of the kernel.  The row stage is scaled by 1 / (N/2), a power
// of two, so that its rounded output cannot exceed the largest gridded value;
// the kernel multiplies |Y|^2 back by (N/2)^2 exactly.
moff_status build_mfma_tables(HostPlan& P, std::string* why) {
  const int N = P.N, L = P.L, NRB = L / 32;
  HostPlan::Mfma& T = P.mfma;
  T.prec = (P.flags & MOFF_MFMA_BF16) ? 2 : 1;
  T.NT = mfma_gather_waves(N) * 64;   // gather lanes
  T.pitch = mfma_layout(N, P.n_taps, P.n_ant).pitch;
  std::vector<int> cells, cost;
  for (int i = 0; i < L * L; ++i) {
    const int n = P.csr_ptr[i + 1] - P.csr_ptr[i];
    if (n > 0) {
      cells.push_back(i);
      cost.push_back(n);
    }
  }
  const long long B = balanced_split(cost, T.NT);
  if (B > (1 << 20)) return fail(why, MOFF_ERR_UNSUPPORTED, "gather program too long");
  if (mfma_layout(N, P.n_taps, P.n_ant).eg > 0xFFFF)
    return fail(why, MOFF_ERR_UNSUPPORTED, "too many antennas and taps for the gather encoding");
  if (mfma_layout(N, P.n_taps, P.n_ant).prog > kMfmaLdsMax)
    return fail(why, MOFF_ERR_UNSUPPORTED, "too many antennas for the matrix-core kernel's LDS");
  T.prog_len = static_cast<int>(B);
  const MfmaLayout lay = mfma_layout(N, P.n_taps, P.n_ant);
  T.grid_base = lay.eg;
  // entry: x = byte offset of e[ant] | byte offset of K[tap] << 16; y = byte
  // address of the cell's real part on the last entry of a cell, else 0
  auto xword = [&](int ant, int tap) {
    return static_cast<uint32_t>(lay.e + 8 * ant) | (static_cast<uint32_t>(lay.k + 8 * tap) << 16);
  };
  T.prog.assign(static_cast<size_t>(T.prog_len) * T.NT, GatherEntry{xword(P.n_ant, 0), 0});
  int lane = 0, k = 0;
  long long cur = 0;
  for (size_t ci = 0; ci < cells.size(); ++ci) {
    if (cur + cost[ci] > B) {
      ++lane;
      k = 0;
      cur = 0;
    }
    cur += cost[ci];
    const int iy = cells[ci] / L, ix = cells[ci] % L;
    for (int e = P.csr_ptr[cells[ci]]; e < P.csr_ptr[cells[ci] + 1]; ++e) {
      T.prog[static_cast<size_t>(k) * T.NT + lane] = GatherEntry{xword(P.csr_ant[e], P.csr_tap[e]), 0};
      ++k;
    }
    T.prog[static_cast<size_t>(k - 1) * T.NT + lane].y = static_cast<uint32_t>(lay.eg + 2 * (iy * T.pitch + ix));
  }

  // [stage][base block][half][k-step][part][lane][slot]: stage 0 = row
  // transform, the B operand W[ix][q] at contraction index
  // ix = 32 k-step + 8 (lane / 16) + slot and column q = 32 block + 16 half +
  // lane % 16; stage 1 = column transform, the A operand V[r][iy] at row
  // r = 32 block + 16 half + lane % 16 and iy likewise.  Part 0 holds the real,
  // part 1 the imaginary part; at q = 0 (r = 0) they hold the real phase
  // vectors of q - N/2 = -N/2 and of q - N/2 = 0.
  const int KS2 = L / 32;
  auto enc = [&](double v) { return T.prec == 2 ? to_bfloat16(v) : to_binary16(v); };
  T.dft.assign(static_cast<size_t>(2) * NRB * 2 * KS2 * 2 * 64 * 8, 0);
  const double s1 = 1.0 / L;
  for (int st = 0; st < 2; ++st)
    for (int b = 0; b < NRB; ++b)
      for (int hf = 0; hf < 2; ++hf)
        for (int ks = 0; ks < KS2; ++ks)
          for (int part = 0; part < 2; ++part)
            for (int ln = 0; ln < 64; ++ln)
              for (int i = 0; i < 8; ++i) {
                const int j = 32 * ks + 8 * (ln / 16) + i;    // ix (stage 0) or iy (stage 1)
                const int n = 32 * b + 16 * hf + ln % 16;     // base column q (stage 0) or row r (stage 1)
                std::complex<double> f;
                if (n == 0)
                  f = std::complex<double>(unit_root(static_cast<long long>(j) * (-L), N).real(), 1.0);
                else
                  f = unit_root(static_cast<long long>(j) * (n - L), N);
                if (st == 0) f *= s1;
                const double v = part == 0 ? f.real() : f.imag();
                T.dft[(((((static_cast<size_t>(st) * NRB + b) * 2 + hf) * KS2 + ks) * 2 + part) * 64 + ln) * 8 + i] =
                    enc(v);
              }
  return MOFF_OK;
}

// Whole antennas to lanes for the fused adjoint's degridding: longest tables
// first, each to the least-loaded lane with a free slot (ties: lowest lane).
// Leaves `slots` empty when some antenna finds no free slot.
void build_adjoint_slots(const HostPlan& P, int NT, std::vector<uint32_t>* slots) {
  slots->clear();
  if (P.n_ant > NT * kAdjSlots) return;
  std::vector<int> order(P.n_ant);
  std::iota(order.begin(), order.end(), 0);
  auto taps = [&](int a) { return P.ktype_k[P.ant_ktype[a]] * P.ktype_k[P.ant_ktype[a]]; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return taps(x) > taps(y); });
  std::vector<long long> load(NT, 0);
  std::vector<int> used(NT, 0);
  std::vector<uint32_t> out(static_cast<size_t>(NT) * kAdjSlots * 2, 0);
  for (size_t i = 0; i < out.size(); i += 2) out[i] = kAdjEmpty;
  for (int a : order) {
    int best = -1;
    for (int l = 0; l < NT; ++l)
      if (used[l] < kAdjSlots && (best < 0 || load[l] < load[best])) best = l;
    if (best < 0) return;
    const int p = P.ant_ktype[a], k = P.ktype_k[p];
    const size_t at = (static_cast<size_t>(best) * kAdjSlots + used[best]) * 2;
    out[at] = static_cast<uint32_t>(a) | (static_cast<uint32_t>(P.ktype_off[p]) << 12) |
              (static_cast<uint32_t>(k) << 24);
    out[at + 1] = static_cast<uint32_t>(P.ix0[a]) | (static_cast<uint32_t>(P.iy0[a]) << 16);
    used[best]++;
    load[best] += taps(a);
  }
  *slots = std::move(out);
}

}  // namespace

uint16_t to_binary16(double x) {
  const uint16_t sign = std::signbit(x) ? 0x8000u : 0u;
  double q = round_sig(std::fabs(x), 11, -24);
  if (!(q < 65520.0)) return static_cast<uint16_t>(sign | 0x7C00u);   // overflow to infinity
  if (q == 0.0) return sign;
  int e = 0;
  (void)std::frexp(q, &e);                  // q = m 2^e
  if (e - 1 < -14)                          // subnormal: q = mant 2^-24
    return static_cast<uint16_t>(sign | static_cast<uint16_t>(std::ldexp(q, 24)));
  const uint16_t mant = static_cast<uint16_t>(std::ldexp(q, 11 - e) - 1024.0);
  return static_cast<uint16_t>(sign | ((e - 1 + 15) << 10) | mant);
}

uint16_t to_bfloat16(double x) {
  // 8 significant bits, float32 exponent range (values here are at most 1 in
  // magnitude, far from overflow); the rounded value is exact in float32.
  const double q = round_sig(std::fabs(x), 8, -133);
  float f = static_cast<float>(std::signbit(x) ? -q : q);
  uint32_t bits = 0;
  std::memcpy(&bits, &f, sizeof(bits));
  return static_cast<uint16_t>(bits >> 16);
}

moff_status build_host_plan(const moff_geometry* g, HostPlan* hp, std::string* why) {
  if (!g || !hp) return fail(why, MOFF_ERR_INVALID_ARG, "null geometry or plan");
  if (g->n_ant < 2 || g->n_ant > kMaxAnt) return fail(why, MOFF_ERR_INVALID_ARG, "n_ant out of [2, 4000]");
  if (!g->ant_xy_m || !g->ktype_k || !g->ktype_vals || !g->ant_ktype || !g->freq_hz)
    return fail(why, MOFF_ERR_INVALID_ARG, "null geometry array");
  if (g->n_ktypes < 1 || g->n_ktypes > kMaxTypes) return fail(why, MOFF_ERR_INVALID_ARG, "n_ktypes out of [1, 4]");
  if (g->n_chan < 1) return fail(why, MOFF_ERR_INVALID_ARG, "n_chan < 1");
  if (g->flags &
      ~uint32_t(MOFF_IN_CI4 | MOFF_AUTOCORR_NONE | MOFF_NORM_PAIRS | MOFF_MFMA_F16 | MOFF_MFMA_BF16 | MOFF_AUTOCORR_UV))
    return fail(why, MOFF_ERR_INVALID_ARG, "unknown flag bits");
  if ((g->flags & MOFF_AUTOCORR_NONE) && (g->flags & MOFF_AUTOCORR_UV))
    return fail(why, MOFF_ERR_INVALID_ARG, "MOFF_AUTOCORR_NONE and MOFF_AUTOCORR_UV exclude each other");
  if ((g->flags & MOFF_MFMA_F16) && (g->flags & MOFF_MFMA_BF16))
    return fail(why, MOFF_ERR_INVALID_ARG, "at most one of MOFF_MFMA_F16 and MOFF_MFMA_BF16");
  if (!is_pow2(g->grid_n) || g->grid_n < 8 || g->grid_n > 256)
    return fail(why, MOFF_ERR_GRID_NOT_POW2, "grid_n must be a power of two in [8, 256]");
  if ((g->flags & (MOFF_MFMA_F16 | MOFF_MFMA_BF16)) && g->grid_n != 64 && g->grid_n != 128)
    return fail(why, MOFF_ERR_UNSUPPORTED, "the MFMA transform is built for grid_n 64 and 128");
  if (!(g->cell_m >= 0.0) || !std::isfinite(g->cell_m)) return fail(why, MOFF_ERR_INVALID_ARG, "bad cell_m");

  HostPlan& P = *hp;
  P = HostPlan{};
  P.n_ant = g->n_ant;
  P.n_ktypes = g->n_ktypes;
  P.n_chan = g->n_chan;
  P.N = g->grid_n;
  P.L = g->grid_n / 2;
  P.flags = g->flags;

  P.ktype_k.assign(g->ktype_k, g->ktype_k + g->n_ktypes);
  P.ktype_off.resize(g->n_ktypes);
  int off = 0;
  for (int p = 0; p < g->n_ktypes; ++p) {
    int k = P.ktype_k[p];
    if (k < 1 || k > kMaxK) return fail(why, MOFF_ERR_INVALID_ARG, "kernel side out of [1, 15]");
    P.ktype_off[p] = off;
    off += k * k;
  }
  P.n_taps = off;
  P.kvals.assign(g->ktype_vals, g->ktype_vals + 2 * off);
  for (float v : P.kvals)
    if (!std::isfinite(v)) return fail(why, MOFF_ERR_INVALID_ARG, "non-finite kernel value");

  P.ant_xy.assign(g->ant_xy_m, g->ant_xy_m + 2 * g->n_ant);
  for (double v : P.ant_xy)
    if (!std::isfinite(v)) return fail(why, MOFF_ERR_INVALID_ARG, "non-finite antenna position");
  P.ant_ktype.assign(g->ant_ktype, g->ant_ktype + g->n_ant);
  for (int t : P.ant_ktype)
    if (t < 0 || t >= g->n_ktypes) return fail(why, MOFF_ERR_INVALID_ARG, "ant_ktype out of range");
  P.freq_hz.assign(g->freq_hz, g->freq_hz + g->n_chan);
  for (double f : P.freq_hz)
    if (!(f > 0.0) || !std::isfinite(f)) return fail(why, MOFF_ERR_INVALID_ARG, "bad frequency");

  // ---- cell size: the default rule (half the shortest wavelength, widened to fit)
  int kmax = 0;
  for (int a = 0; a < P.n_ant; ++a) kmax = std::max(kmax, P.ktype_k[P.ant_ktype[a]]);
  if (g->cell_m > 0.0) {
    P.cell_m = g->cell_m;
  } else {
    double fmax = *std::max_element(P.freq_hz.begin(), P.freq_hz.end());
    double lam_min = kC / fmax;
    double xmin = P.ant_xy[0], xmax = P.ant_xy[0], ymin = P.ant_xy[1], ymax = P.ant_xy[1];
    for (int a = 1; a < P.n_ant; ++a) {
      xmin = std::min(xmin, P.ant_xy[2 * a]);
      xmax = std::max(xmax, P.ant_xy[2 * a]);
      ymin = std::min(ymin, P.ant_xy[2 * a + 1]);
      ymax = std::max(ymax, P.ant_xy[2 * a + 1]);
    }
    double span = std::max(xmax - xmin, ymax - ymin);
    int room = P.L - kmax - 1;
    if (room <= 0) return fail(why, MOFF_ERR_FOOTPRINT_OVERFLOW, "grid too small for the largest footprint");
    P.cell_m = std::max(lam_min / 2.0, span / static_cast<double>(room));
  }

  // ---- footprint lower-left cells: floor(x / cell - (k - 1) / 2 + 0.5), shifted to start at 0
  P.ix0.resize(P.n_ant);
  P.iy0.resize(P.n_ant);
  std::vector<long long> ix(P.n_ant), iy(P.n_ant);
  for (int a = 0; a < P.n_ant; ++a) {
    double h = (static_cast<double>(P.ktype_k[P.ant_ktype[a]]) - 1.0) / 2.0;
    double fx = std::floor(P.ant_xy[2 * a] / P.cell_m - h + 0.5);
    double fy = std::floor(P.ant_xy[2 * a + 1] / P.cell_m - h + 0.5);
    if (std::fabs(fx) > 1e15 || std::fabs(fy) > 1e15)
      return fail(why, MOFF_ERR_FOOTPRINT_OVERFLOW, "antenna far outside the grid");
    ix[a] = static_cast<long long>(fx);
    iy[a] = static_cast<long long>(fy);
  }
  long long mx = *std::min_element(ix.begin(), ix.end());
  long long my = *std::min_element(iy.begin(), iy.end());
  for (int a = 0; a < P.n_ant; ++a) {
    long long k = P.ktype_k[P.ant_ktype[a]];
    long long x0 = ix[a] - mx, y0 = iy[a] - my;
    if (x0 + k > P.L || y0 + k > P.L)
      return fail(why, MOFF_ERR_FOOTPRINT_OVERFLOW, "footprints extend beyond the N/2 aperture region");
    P.ix0[a] = static_cast<int32_t>(x0);
    P.iy0[a] = static_cast<int32_t>(y0);
  }
  P.lm_per_pixel.resize(P.n_chan);
  for (int c = 0; c < P.n_chan; ++c) P.lm_per_pixel[c] = (kC / P.freq_hz[c]) / (P.N * P.cell_m);

  // ---- CSR keyed by aperture cell (stable counting sort: antenna-ascending within a cell).
  // Table entries that are exactly zero contribute nothing to the gridded field
  // and are left out (the corners of a tapered table, for instance).
  const int L = P.L, N = P.N;
  auto tap_nonzero = [&](int tap) { return P.kvals[2 * tap] != 0.0 || P.kvals[2 * tap + 1] != 0.0; };
  P.csr_ptr.assign(L * L + 1, 0);
  for (int a = 0; a < P.n_ant; ++a) {
    int p = P.ant_ktype[a], k = P.ktype_k[p];
    for (int u = 0; u < k; ++u)
      for (int v = 0; v < k; ++v)
        if (tap_nonzero(P.ktype_off[p] + u * k + v)) P.csr_ptr[(P.iy0[a] + u) * L + (P.ix0[a] + v) + 1]++;
  }
  for (int i = 0; i < L * L; ++i) P.csr_ptr[i + 1] += P.csr_ptr[i];
  P.csr_ant.resize(P.csr_ptr[L * L]);
  P.csr_tap.resize(P.csr_ptr[L * L]);
  {
    std::vector<int32_t> fill(P.csr_ptr.begin(), P.csr_ptr.end() - 1);
    for (int a = 0; a < P.n_ant; ++a) {
      int p = P.ant_ktype[a], k = P.ktype_k[p];
      for (int u = 0; u < k; ++u)
        for (int v = 0; v < k; ++v) {
          const int tap = P.ktype_off[p] + u * k + v;
          if (!tap_nonzero(tap)) continue;
          int cell = (P.iy0[a] + u) * L + (P.ix0[a] + v);
          int at = fill[cell]++;
          P.csr_ant[at] = a;
          P.csr_tap[at] = tap;
        }
    }
  }

  // ---- power patterns |DFT_N(K_p)|^2 in float64 (same sign and origin as the image)
  P.Pp.assign(static_cast<size_t>(P.n_ktypes) * N * N, 0.0);
  for (int p = 0; p < P.n_ktypes; ++p) {
    int k = P.ktype_k[p];
    std::vector<std::complex<double>> K(k * k), A(static_cast<size_t>(N) * k), B(static_cast<size_t>(N) * k);
    for (int i = 0; i < k * k; ++i)
      K[i] = {P.kvals[2 * (P.ktype_off[p] + i)], P.kvals[2 * (P.ktype_off[p] + i) + 1]};
    for (int r = 0; r < N; ++r)
      for (int u = 0; u < k; ++u) A[r * k + u] = unit_root(static_cast<long long>(u) * (r - N / 2), N);
    // B[r][v] = sum_u A[r][u] K[u][v]
    for (int r = 0; r < N; ++r)
      for (int v = 0; v < k; ++v) {
        std::complex<double> s = 0;
        for (int u = 0; u < k; ++u) s += A[r * k + u] * K[u * k + v];
        B[r * k + v] = s;
      }
    double* out = &P.Pp[static_cast<size_t>(p) * N * N];
    for (int r = 0; r < N; ++r)
      for (int q = 0; q < N; ++q) {
        std::complex<double> s = 0;
        for (int v = 0; v < k; ++v) s += B[r * k + v] * A[q * k + v];
        out[r * N + q] = std::norm(s);
      }
  }

  // ---- uv-plane rule: power patterns summed over antennas, table autocorrelation at zero lag
  {
    std::vector<int> count(P.n_ktypes, 0);
    for (int a = 0; a < P.n_ant; ++a) count[P.ant_ktype[a]]++;
    P.Pn.assign(static_cast<size_t>(N) * N, 0.0);
    P.a0 = 0.0;
    for (int p = 0; p < P.n_ktypes; ++p) {
      double e2 = 0.0;
      const int kk = P.ktype_k[p] * P.ktype_k[p];
      for (int i = 0; i < kk; ++i) {
        const double re = P.kvals[2 * (P.ktype_off[p] + i)], im = P.kvals[2 * (P.ktype_off[p] + i) + 1];
        e2 += re * re + im * im;
      }
      P.a0 += count[p] * e2;
      const double* src = &P.Pp[static_cast<size_t>(p) * N * N];
      for (size_t i = 0; i < static_cast<size_t>(N) * N; ++i) P.Pn[i] += count[p] * src[i];
    }
    if (!(P.a0 > 0.0) && (g->flags & MOFF_AUTOCORR_UV))
      return fail(why, MOFF_ERR_INVALID_ARG, "MOFF_AUTOCORR_UV needs a nonzero illumination table");
  }

  // ---- twiddles
  P.twiddle.resize(2 * N);
  for (int k = 0; k < N; ++k) {
    std::complex<double> w = unit_root(k, N);
    P.twiddle[2 * k] = static_cast<float>(w.real());
    P.twiddle[2 * k + 1] = static_cast<float>(w.imag());
  }

  // ---- fused frame transform: folded-grid gather programs, per shape variant and column class w
  for (int v = 0; v < kMaxVariants; ++v) {
    const FrameShape S = frame_shape(N, v);
    if (S.N != N) continue;
    HostPlan::Variant V;
    V.shape = S;
    V.n_taps_ = P.n_taps;
    V.M = N / S.SX;
    V.NZR = std::min(L, V.M);
    V.NJ = std::max(1, L / V.M);
    V.ZP = grid_pitch(V.M);
    if (V.NJ * P.n_taps >= 2048) return fail(why, MOFF_ERR_UNSUPPORTED, "too many kernel taps for the gather encoding");
    V.weights.assign(static_cast<size_t>(2) * S.SX * V.NJ * P.n_taps, 0.f);
    for (int w = 0; w < S.SX; ++w)
      for (int j = 0; j < V.NJ; ++j) {
        std::complex<double> rot = unit_root(static_cast<long long>(j) * w, S.SX);
        for (int t = 0; t < P.n_taps; ++t) {
          std::complex<double> kv(P.kvals[2 * t], P.kvals[2 * t + 1]);
          std::complex<double> wv = kv * rot;
          size_t at = (static_cast<size_t>(w) * V.NJ * P.n_taps + j * P.n_taps + t) * 2;
          V.weights[at] = static_cast<float>(wv.real());
          V.weights[at + 1] = static_cast<float>(wv.imag());
        }
      }

    // The fused transform runs on the transposed aperture: folded-grid row a is
    // aperture column ix = a, and the folded axis runs along y, so a workgroup's
    // output class is a residue class of image rows and it writes whole image
    // rows.  Folded cells (a, n'), n' < NZR, row-major; entries from aperture
    // cells (iy, ix) = (n' + j M, a), j ascending, antenna ascending within a
    // cell.  Every folded cell is written every frame (an empty one by a single
    // entry that reads the all-zero antenna slot).
    auto csr_cell = [&](int a, int m) { return m * L + a; };   // CSR index of aperture cell (iy = m, ix = a)
    const int ncell = L * V.NZR;
    std::vector<int> cost(ncell);
    int maxc = 0;
    for (int a = 0; a < L; ++a)
      for (int n = 0; n < V.NZR; ++n) {
        int c = 0;
        for (int j = 0; j < V.NJ; ++j) {
          int m = n + j * V.M;
          if (m < L) c += P.csr_ptr[csr_cell(a, m) + 1] - P.csr_ptr[csr_cell(a, m)];
        }
        maxc = std::max(maxc, c);
        cost[a * V.NZR + n] = std::max(1, c);
      }
    P.max_cell_entries = maxc;
    // Lanes take contiguous runs of cells, split greedily by cost.  A segment
    // is a range of cells split over a range of lanes.
    struct Segment {
      std::vector<std::pair<int, int>> runs;   // cell ranges [begin, end), a lane never spans two
      int lane0, lanes;
    };
    // smallest per-lane load B for which the greedy split of a segment needs
    // no more than its lanes
    auto min_load = [&](const Segment& g) {
      auto lanes_needed = [&](long long B) {
        int lanes = 0;
        for (const auto& run : g.runs) {
          if (run.first >= run.second) continue;
          ++lanes;
          long long cur = 0;
          for (int i = run.first; i < run.second; ++i) {
            if (cur + cost[i] > B) {
              ++lanes;
              cur = 0;
            }
            cur += cost[i];
          }
        }
        return lanes;
      };
      long long lo = 0, hi = 0;
      for (const auto& run : g.runs)
        for (int i = run.first; i < run.second; ++i) {
          lo = std::max<long long>(lo, cost[i]);
          hi += cost[i];
        }
      while (lo < hi) {
        long long mid = (lo + hi) / 2;
        if (lanes_needed(mid) <= g.lanes) hi = mid;
        else lo = mid + 1;
      }
      return lo;
    };
    std::vector<Segment> segs{Segment{{{0, ncell}}, 0, S.NT}};
    long long B = min_load(segs[0]);
    // Wave-owned rows: when one step of the row stage covers every folded row,
    // each wave can grid exactly the rows it transforms (stage_row); the
    // kernel then needs no workgroup barrier between the gather and the row
    // stage.  Taken when the per-wave split lengthens the program by at most
    // 1/8 (the densest wave sets the length).
    const int NW = S.NT / 64, RPW = 64 / row_lanes(S);
    V.wave_rows = false;
    if (NW > 1 && NW * RPW == L) {
      std::vector<Segment> ws;
      long long Bw = 0;
      for (int w = 0; w < NW; ++w) {
        Segment g{{}, 64 * w, 64};
        for (int r = 0; r < RPW; ++r) {
          const int row = stage_row(S, 0, w, r);
          if (!g.runs.empty() && g.runs.back().second == row * V.NZR) g.runs.back().second += V.NZR;
          else g.runs.push_back({row * V.NZR, (row + 1) * V.NZR});
        }
        Bw = std::max(Bw, min_load(g));
        ws.push_back(std::move(g));
      }
      if (8 * Bw <= 9 * B) {
        segs = ws;
        B = Bw;
        V.wave_rows = true;
      }
    }
    V.prog_len = static_cast<int>((B + 3) / 4 * 4);
    if (V.prog_len > (1 << 20)) return fail(why, MOFF_ERR_UNSUPPORTED, "gather program too long");
    const uint32_t zero_slot = static_cast<uint32_t>(P.n_ant);
    V.prog.assign(static_cast<size_t>(S.SX) * V.prog_len * S.NT, GatherEntry{zero_slot, 0});
    V.cell0.assign(static_cast<size_t>(S.SX) * S.NT, 0);
    for (int w = 0; w < S.SX; ++w) {
     for (const Segment& g : segs) {
      GatherEntry* base = &V.prog[static_cast<size_t>(w) * V.prog_len * S.NT];
      int lane = g.lane0 - 1, k = 0;
      long long cur = 0;
      for (const auto& run : g.runs) {
       if (run.first >= run.second) continue;
       ++lane;
       k = 0;
       cur = 0;
       V.cell0[static_cast<size_t>(w) * S.NT + lane] = run.first;
       for (int i = run.first; i < run.second; ++i) {
        if (cur + cost[i] > B) {
          ++lane;
          k = 0;
          cur = 0;
          V.cell0[static_cast<size_t>(w) * S.NT + lane] = i;
        }
        cur += cost[i];
        const int a = i / V.NZR, n = i % V.NZR;
        const uint32_t dst = static_cast<uint32_t>(a * V.ZP + n);
        int emitted = 0;
        for (int j = 0; j < V.NJ; ++j) {
          int m = n + j * V.M;
          if (m >= L) continue;
          for (int e = P.csr_ptr[csr_cell(a, m)]; e < P.csr_ptr[csr_cell(a, m) + 1]; ++e) {
            uint32_t wi = static_cast<uint32_t>(j * P.n_taps + P.csr_tap[e]);
            base[static_cast<size_t>(k) * S.NT + lane] = GatherEntry{static_cast<uint32_t>(P.csr_ant[e]) | (wi << 12), dst};
            ++k;
            ++emitted;
          }
        }
        if (emitted == 0) {
          base[static_cast<size_t>(k) * S.NT + lane] = GatherEntry{zero_slot, dst};
          ++k;
        }
        base[static_cast<size_t>(k - 1) * S.NT + lane].x |= kStoreBit;
       }
      }
     }
    }
    // device form: x words, four consecutive entries of a lane side by side
    V.prog4.assign(V.prog.size(), zero_slot);
    const int K4 = V.prog_len / 4;
    for (int w = 0; w < S.SX; ++w)
      for (int k = 0; k < V.prog_len; ++k)
        for (int lane = 0; lane < S.NT; ++lane)
          V.prog4[((static_cast<size_t>(w) * K4 + k / 4) * S.NT + lane) * 4 + k % 4] =
              V.prog[(static_cast<size_t>(w) * V.prog_len + k) * S.NT + lane].x;
    // real weights: each entry's weight next to it (the all-zero slot's entries get 0)
    bool real = true;
    for (size_t i = 1; i < V.weights.size(); i += 2) real = real && V.weights[i] == 0.f;
    if (real) {
      V.progw.assign(V.prog4.size(), 0.f);
      for (size_t i = 0; i < V.prog4.size(); ++i) {
        const uint32_t x = V.prog4[i];
        const int w = static_cast<int>(i / (static_cast<size_t>(K4) * S.NT * 4));
        const uint32_t wi = (x >> 12) & 0x7FFu;
        V.progw[i] = (x & 0xFFFu) == zero_slot ? 0.f : V.weights[(static_cast<size_t>(w) * V.n_weights() + wi) * 2];
      }
    }
    // Destination-carrying entries (device form, real weights only): when the
    // folded grid takes more than half a CU's LDS, one workgroup runs per CU
    // and nothing hides the gather's per-cell store branch, so each entry
    // instead carries its cell's LDS element and a "first entry of the cell"
    // flag, and every entry stores its cell's running sum (the cell's last
    // entry stores the final one): x = slot | element << 12 | first << 30.
    // Padding entries (the zero slot) write to the unused pad column of row 0.
    V.dst_entries = real && sizeof(float) * 2 * static_cast<size_t>(L) * V.ZP > 80u * 1024;
    if (V.dst_entries) {
      const uint32_t pad_elem = static_cast<uint32_t>(V.ZP - 1);
      if (static_cast<size_t>(L) * V.ZP > (1u << 16)) return fail(why, MOFF_ERR_UNSUPPORTED, "grid too large for the entry form");
      for (int w = 0; w < S.SX; ++w)
        for (int lane = 0; lane < S.NT; ++lane) {
          bool first = true;
          for (int k = 0; k < V.prog_len; ++k) {
            const GatherEntry& ge = V.prog[(static_cast<size_t>(w) * V.prog_len + k) * S.NT + lane];
            const bool pad = (ge.x & 0xFFFu) == zero_slot && ge.y == 0 && !(ge.x & kStoreBit);
            V.prog4[((static_cast<size_t>(w) * K4 + k / 4) * S.NT + lane) * 4 + k % 4] =
                (ge.x & 0xFFFu) | ((pad ? pad_elem : ge.y) << 12) | ((first && !pad) ? kFirstBit : 0u);
            first = (ge.x & kStoreBit) != 0;
          }
        }
    }
    build_adjoint_slots(P, S.NT, &V.slots);
    P.variants.push_back(std::move(V));
  }
  if (P.variants.empty()) return fail(why, MOFF_ERR_UNSUPPORTED, "no frame shape for this grid size");
  if (P.flags & (MOFF_MFMA_F16 | MOFF_MFMA_BF16)) {
    moff_status s = build_mfma_tables(P, why);
    if (s != MOFF_OK) return s;
  }
  return MOFF_OK;
}

}  // namespace moff
