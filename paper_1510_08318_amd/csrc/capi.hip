// C ABI of the MOFF library (declared in include/moff.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/moff.h"
#include "fx.h"
#include "fx_tables.h"
#include "kernels.h"
#include "plan.h"

using moff::GatherEntry;
using moff::HostPlan;

struct moff_plan_s {
  HostPlan hp;
  int device = -1;
  // device tables
  uint4* d_prog[moff::kMaxVariants] = {};       // HostPlan::Variant::prog4
  float4* d_progw[moff::kMaxVariants] = {};     // HostPlan::Variant::progw (null: complex weights)
  int* d_cell0[moff::kMaxVariants] = {};
  float2* d_weights[moff::kMaxVariants] = {};
  float2* d_tw = nullptr;
  double* d_Pp = nullptr;
  int* d_ant_type = nullptr;
  float2* d_ktab = nullptr;
  int* d_csr_ptr = nullptr;
  int* d_csr_ant = nullptr;
  int* d_csr_tap = nullptr;
  int* d_ant_cells = nullptr;   // [n_ant][2] (ix0, iy0)
  int* d_ktype_k = nullptr;
  int* d_ktype_off = nullptr;
  GatherEntry* d_mfma_prog = nullptr;   // reduced-precision path (MOFF_MFMA_*)
  uint16_t* d_mfma_dft = nullptr;
  double* d_Pn = nullptr;               // uv-plane autocorrelation rule (MOFF_AUTOCORR_UV)
  uint32_t* d_adj_slots[moff::kMaxVariants] = {};   // fused adjoint: antennas per lane; null if they do not fit
  // visibility route (moff_image_fx), built on first use
  int* d_fx_ptr = nullptr;
  int* d_fx_ab = nullptr;
  float2* d_fx_x = nullptr;
  int fx_NL = 0, fx_xs = 0;
  // workspace, grown on demand
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  void* d_aux = nullptr;                // S / A or shifted sensitivities of the uv rule
  size_t aux_bytes = 0;
  // optional kernel timing
  bool timing = false, timed = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // fused launch configuration (heuristic default, or chosen by the autotuner)
  int cu_count = 0;
  int variant = 0;          // index into hp.variants
  int slices = 0;           // time slices; 0 = heuristic
  bool tuned = false;
  int adj_waves = 1;        // fused adjoint: waves per SIMD its registers are sized for
  int adj_variant = 0;      // fused adjoint: shape variant (set with the image's, or tuned on its own)
};

namespace {

// Fixed device scratch of moff_image_noalloc (for callers that cannot
// allocate): the per-slice partial sums and float64 running sums of its fused
// call.  Each GPU the library runs on holds its own copy until the process
// ends.  Host code never passes this name to a kernel: it is a host-side
// stand-in, and the device address of each GPU's copy comes from
// hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[MOFF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current: looked up
// once per device (at plan creation) and kept.
moff_status noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return MOFF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MOFF_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MOFF_OK;
}

// Run f with the plan's device current, restoring the caller's device after.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    ok_ = hipGetDevice(&prev_) == hipSuccess;
    if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    switched_ = ok_ && prev_ != dev;
  }
  ~DeviceGuard() {
    if (switched_) (void)hipSetDevice(prev_);
  }
  bool ok() const { return ok_; }

 private:
  int prev_ = 0;
  bool ok_ = false, switched_ = false;
};

template <class T>
moff_status upload(T** dst, const void* src, size_t bytes) {
  if (bytes == 0) bytes = sizeof(T);
  if (hipMalloc(reinterpret_cast<void**>(dst), bytes) != hipSuccess) return MOFF_ERR_NOMEM;
  if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return MOFF_ERR_HIP;
  return MOFF_OK;
}

void free_device(moff_plan p) {
  void* ptrs[] = {p->d_tw,        p->d_Pp,        p->d_ant_type, p->d_ktab,        p->d_csr_ptr,
                  p->d_csr_ant,   p->d_csr_tap,   p->d_ant_cells, p->d_ktype_k,    p->d_ktype_off,
                  p->d_mfma_prog, p->d_mfma_dft,  p->d_Pn,        p->d_ws,         p->d_aux,
                  p->d_fx_ptr,    p->d_fx_ab,     p->d_fx_x};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (int v = 0; v < moff::kMaxVariants; ++v) {
    if (p->d_prog[v]) (void)hipFree(p->d_prog[v]);
    if (p->d_cell0[v]) (void)hipFree(p->d_cell0[v]);
    if (p->d_progw[v]) (void)hipFree(p->d_progw[v]);
    if (p->d_adj_slots[v]) (void)hipFree(p->d_adj_slots[v]);
    if (p->d_weights[v]) (void)hipFree(p->d_weights[v]);
  }
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
}

// Grow a plan-owned device buffer to at least `bytes` (contents are not kept;
// the device is synchronised before an old buffer is released).
moff_status grow(void** buf, size_t* have, size_t bytes) {
  if (bytes <= *have) return MOFF_OK;
  if (*buf) {
    (void)hipDeviceSynchronize();
    (void)hipFree(*buf);
    *buf = nullptr;
    *have = 0;
  }
  if (hipMalloc(buf, bytes) != hipSuccess) return MOFF_ERR_NOMEM;
  *have = bytes;
  return MOFF_OK;
}

moff_status ensure_workspace(moff_plan p, size_t bytes) { return grow(&p->d_ws, &p->ws_bytes, bytes); }
moff_status ensure_aux(moff_plan p, size_t bytes) { return grow(&p->d_aux, &p->aux_bytes, bytes); }

moff_status hip_status(hipError_t e) { return e == hipSuccess ? MOFF_OK : MOFF_ERR_HIP; }

bool uv_rule(const HostPlan& hp) { return (hp.flags & MOFF_AUTOCORR_UV) != 0; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

moff_status check_compute(moff_plan p, int64_t n_time) {
  if (!p) return MOFF_ERR_INVALID_ARG;
  if (p->device < 0) return MOFF_ERR_UNSUPPORTED;
  if (n_time < 1) return MOFF_ERR_INVALID_ARG;
  if (n_time * static_cast<int64_t>(p->hp.n_chan) >= (int64_t(1) << 31)) return MOFF_ERR_UNSUPPORTED;
  return MOFF_OK;
}

double image_scale(const HostPlan& hp, int64_t n_time) {
  double s = 1.0 / static_cast<double>(n_time);
  if (hp.flags & MOFF_NORM_PAIRS) s /= static_cast<double>(hp.n_ant) * (hp.n_ant - 1);
  return s;
}

// The uv-plane rule on accumulated sums S [C][N][N] (Sec. 4.2), into `image`.
moff_status uv_finalize(moff_plan p, const float* S, int64_t n_time, float* image, hipStream_t st) {
  const HostPlan& hp = p->hp;
  moff::UvArgs u{};
  u.S = S;
  u.Pn = p->d_Pn;
  u.out = image;
  u.N = hp.N;
  u.n_chan = hp.n_chan;
  u.a0 = hp.a0;
  u.scale = image_scale(hp, n_time);
  return hip_status(moff::launch_uv_finalize(u, st));
}

struct LaunchConfig {
  int variant, slices, grid;
};

constexpr int kTuneReps = 3;    // timed batches per autotuner candidate
constexpr int kTuneBatch = 3;   // back-to-back calls per timed batch (steady state, as in use)
constexpr float kTuneSlack = 0.03f;   // calls this much slower than the fastest still count as equal

bool is_mfma(const HostPlan& hp) { return hp.mfma.prec != 0; }

// Work items per time slice, LDS bytes and resident workgroups of a variant.
struct KernelFootprint {
  int per_slice;
  size_t lds;
  int resident;
  int threads;
};

KernelFootprint footprint(moff_plan p, int variant) {
  const HostPlan& hp = p->hp;
  const bool ci4 = hp.flags & MOFF_IN_CI4;
  KernelFootprint f{};
  if (is_mfma(hp)) {
    f.per_slice = hp.n_chan;
    const bool in_lds = moff::mfma_prog_in_lds(hp.N, hp.n_taps, hp.n_ant, hp.mfma.prog_len);
    f.lds = moff::mfma_lds_bytes(hp.N, hp.n_taps, hp.n_ant, hp.mfma.prog_len, in_lds);
    f.resident = std::max(1, moff::mfma_blocks_per_cu(hp.N, hp.mfma.prec, ci4, f.lds)) * std::max(1, p->cu_count);
    f.threads = moff::mfma_threads(hp.N);
  } else {
    const HostPlan::Variant& V = hp.variants[variant];
    f.per_slice = V.shape.SX * hp.n_chan;
    f.lds = moff::fused_lds_bytes(hp.N, variant, V.n_weights(), hp.n_ant);
    f.resident = std::max(1, moff::fused_blocks_per_cu(hp.N, variant, ci4, f.lds)) * std::max(1, p->cu_count);
    f.threads = V.shape.NT;
  }
  return f;
}

int n_variants(const HostPlan& hp) { return is_mfma(hp) ? 1 : static_cast<int>(hp.variants.size()); }

// Workgroups of a fused launch with `slices` time slices.  The float32 kernel
// places the column classes of one (channel, slice) on one XCD and pads the
// (channel, slice) count to a multiple of 8 (moff::kXcds); padding workgroups
// exit at once.
int launch_grid(const HostPlan& hp, int variant, int slices) {
  if (is_mfma(hp)) return hp.n_chan * slices;
  const int cs = hp.n_chan * slices;
  return hp.variants[variant].shape.SX * ((cs + moff::kXcds - 1) / moff::kXcds * moff::kXcds);
}

// Launch configuration for n_time frames: the tuned or set choice, else a
// heuristic: shape variant 0 and enough time slices for about two rounds of
// resident workgroups.  One work item (column class, channel, time slice) per
// workgroup.
LaunchConfig launch_config(moff_plan p, int64_t n_time) {
  const HostPlan& hp = p->hp;
  LaunchConfig lc{};
  lc.variant = std::min<int>(p->variant, n_variants(hp) - 1);
  const KernelFootprint f = footprint(p, lc.variant);
  const int per_slice = f.per_slice, resident = f.resident;
  int slices = p->slices;
  if (slices <= 0) slices = (2 * resident + per_slice - 1) / per_slice;
  slices = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({static_cast<int64_t>(slices), n_time, 256})));
  lc.slices = slices;
  lc.grid = launch_grid(hp, lc.variant, slices);
  return lc;
}

moff::FusedArgs fused_args(moff_plan p, int variant, const void* E, int64_t n_time, const float* gains) {
  const HostPlan& hp = p->hp;
  const HostPlan::Variant& V = hp.variants[variant];
  moff::FusedArgs a{};
  a.E = E;
  a.gains = reinterpret_cast<const float2*>(gains);
  a.prog = p->d_prog[variant];
  a.progw = p->d_progw[variant];
  a.cell0 = p->d_cell0[variant];
  a.prog_len = V.prog_len;
  a.wave_rows = V.wave_rows ? 1 : 0;
  a.dst_entries = V.dst_entries ? 1 : 0;
  a.weights = p->d_weights[variant];
  a.n_weights = V.n_weights();
  a.tw = p->d_tw;
  a.ant_type = p->d_ant_type;
  a.n_ant = hp.n_ant;
  a.n_chan = hp.n_chan;
  a.n_types = hp.n_ktypes;
  a.n_time = n_time;
  a.Pp = p->d_Pp;
  a.subtract = (hp.flags & MOFF_AUTOCORR_NONE) ? 0 : 1;
  return a;
}

moff::MfmaArgs mfma_args(moff_plan p, const void* E, int64_t n_time, const float* gains) {
  const HostPlan& hp = p->hp;
  moff::MfmaArgs a{};
  a.E = E;
  a.gains = reinterpret_cast<const float2*>(gains);
  a.prog = p->d_mfma_prog;
  a.prog_len = hp.mfma.prog_len;
  a.prog_in_lds = moff::mfma_prog_in_lds(hp.N, hp.n_taps, hp.n_ant, hp.mfma.prog_len) ? 1 : 0;
  a.ktab = p->d_ktab;
  a.n_taps = hp.n_taps;
  a.dft = p->d_mfma_dft;
  a.ant_type = p->d_ant_type;
  a.n_ant = hp.n_ant;
  a.n_chan = hp.n_chan;
  a.n_types = hp.n_ktypes;
  a.n_time = n_time;
  a.Pp = p->d_Pp;
  a.subtract = (hp.flags & MOFF_AUTOCORR_NONE) ? 0 : 1;
  return a;
}

// One launch of the plan's fused kernel (float32 FFT or reduced-precision MFMA
// transform) writing `out` / `outA` in epilogue `mode`.
hipError_t launch_fused_kernel(moff_plan p, const LaunchConfig& lc, const void* E, int64_t n_time,
                               const float* gains, float* out, double* outA, int mode, double* run64,
                               hipStream_t st) {
  const HostPlan& hp = p->hp;
  const bool ci4 = hp.flags & MOFF_IN_CI4;
  if (is_mfma(hp)) {
    moff::MfmaArgs a = mfma_args(p, E, n_time, gains);
    a.slices = lc.slices;
    a.scale = image_scale(hp, n_time);
    a.out = out;
    a.outA = outA;
    a.mode = mode;
    return moff::launch_mfma(a, hp.N, hp.mfma.prec, ci4, lc.grid, st);
  }
  moff::FusedArgs a = fused_args(p, lc.variant, E, n_time, gains);
  a.progress_prio = footprint(p, lc.variant).resident > std::max(1, p->cu_count) ? 1 : 0;
  a.slices = lc.slices;
  a.scale = image_scale(hp, n_time);
  a.out = out;
  a.outA = outA;
  a.mode = mode;
  a.acc64 = run64;
  return moff::launch_fused(a, hp.N, lc.variant, ci4, lc.grid, st);
}

// Scratch a fused call needs: per-slice partial sums (more than one slice) and
// the float64 running sums of blocked accumulation (a float32-path slice longer
// than kBlockFrames samples).
struct FusedScratch {
  size_t s_bytes, a_bytes, run_bytes;
  size_t total() const { return s_bytes + a_bytes + run_bytes; }
};

FusedScratch fused_scratch(const HostPlan& hp, const LaunchConfig& lc, int64_t n_time) {
  const size_t pixels = static_cast<size_t>(hp.N) * hp.N * hp.n_chan * lc.slices;
  FusedScratch f{};
  if (lc.slices > 1) {
    f.s_bytes = sizeof(float) * pixels;
    f.a_bytes = sizeof(double) * hp.n_chan * hp.n_ktypes * lc.slices;
  }
  const int64_t longest = (n_time + lc.slices - 1) / lc.slices;
  if (!is_mfma(hp) && longest > moff::kBlockFrames)
    f.run_bytes = sizeof(double) * moff::fused_lane_values(hp.N, lc.variant) * hp.n_chan * lc.slices;
  return f;
}

// One fused call in configuration lc.  Its scratch comes from `scratch`
// (at least fused_scratch(...).total() bytes, 256-byte aligned) or, when that
// is null, from the plan's workspace, grown on demand.
moff_status fused_run_cfg(moff_plan p, const LaunchConfig& lc, const void* E, int64_t n_time, const float* gains,
                          float* out, double* outA, bool final_image, hipStream_t st, void* scratch = nullptr) {
  const HostPlan& hp = p->hp;
  if (footprint(p, lc.variant).lds > size_t(159) * 1024) return MOFF_ERR_UNSUPPORTED;
  const double scale = image_scale(hp, n_time);
  const int subtract = (hp.flags & MOFF_AUTOCORR_NONE) ? 0 : 1;
  const FusedScratch fs = fused_scratch(hp, lc, n_time);
  char* ws = static_cast<char*>(scratch);
  if (!ws && fs.total() > 0) {
    moff_status ms = ensure_workspace(p, fs.total());
    if (ms != MOFF_OK) return ms;
    ws = static_cast<char*>(p->d_ws);
  }
  double* run64 = fs.run_bytes ? reinterpret_cast<double*>(ws + fs.s_bytes + fs.a_bytes) : nullptr;
  if (lc.slices == 1) {
    if (p->timing && hipEventRecord(p->ev0, st) != hipSuccess) return MOFF_ERR_HIP;
    hipError_t e = launch_fused_kernel(p, lc, E, n_time, gains, out, outA,
                                       final_image ? moff::kModeFinal : moff::kModeAccum, run64, st);
    if (e != hipSuccess) return MOFF_ERR_HIP;
    if (p->timing) {
      if (hipEventRecord(p->ev1, st) != hipSuccess) return MOFF_ERR_HIP;
      p->timed = true;
    }
    return MOFF_OK;
  }
  float* S_part = reinterpret_cast<float*>(ws);
  double* A_part = reinterpret_cast<double*>(ws + fs.s_bytes);
  if (p->timing && hipEventRecord(p->ev0, st) != hipSuccess) return MOFF_ERR_HIP;
  hipError_t e = launch_fused_kernel(p, lc, E, n_time, gains, S_part, A_part, moff::kModePartial, run64, st);
  if (e != hipSuccess) return MOFF_ERR_HIP;
  if (p->timing) {
    if (hipEventRecord(p->ev1, st) != hipSuccess) return MOFF_ERR_HIP;
    p->timed = true;
  }
  moff::ReduceArgs r{};
  r.S_part = S_part;
  r.A_part = A_part;
  r.Pp = p->d_Pp;
  r.out = out;
  r.outA = outA;
  r.N = hp.N;
  r.n_chan = hp.n_chan;
  r.n_types = hp.n_ktypes;
  r.slices = lc.slices;
  r.final_image = final_image ? 1 : 0;
  r.subtract = subtract;
  r.scale = scale;
  return hip_status(moff::launch_reduce(r, st));
}

moff_status fused_run(moff_plan p, const void* E, int64_t n_time, const float* gains, float* out, double* outA,
                      bool final_image, hipStream_t st) {
  return fused_run_cfg(p, launch_config(p, n_time), E, n_time, gains, out, outA, final_image, st);
}

moff::GridArgs grid_args(moff_plan p, const void* E, int64_t n_time, const float* gains) {
  const HostPlan& hp = p->hp;
  moff::GridArgs g{};
  g.E = E;
  g.gains = reinterpret_cast<const float2*>(gains);
  g.ktab = p->d_ktab;
  g.csr_ptr = p->d_csr_ptr;
  g.csr_ant = p->d_csr_ant;
  g.csr_tap = p->d_csr_tap;
  g.ant_type = p->d_ant_type;
  g.n_ant = hp.n_ant;
  g.n_chan = hp.n_chan;
  g.n_taps = hp.n_taps;
  g.n_types = hp.n_ktypes;
  g.L = hp.L;
  g.n_time = n_time;
  return g;
}

moff_status gain_vjp(moff_plan p, const void* E, int64_t n_time, const float* gains, const float* dL_dimage,
                     float* dL_dgains, void* stream, bool force_staged) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !dL_dimage || !dL_dgains || !aligned16(dL_dimage) || !aligned16(dL_dgains) ||
      (gains && !aligned16(gains)))
    return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  const HostPlan& hp = p->hp;
  const HostPlan::Variant& V = hp.variants[0];
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool ci4 = hp.flags & MOFF_IN_CI4;
  const size_t npix = static_cast<size_t>(hp.N) * hp.N;
  // Under the uv-plane rule the image is scale * (S - beta Pn) with beta linear in
  // S, so its sensitivities with respect to S are R shifted by <R, Pn> / (N^2 a0)
  // per channel, and no per-antenna term remains.
  const float* R = dL_dimage;
  if (uv_rule(hp)) {
    s = ensure_aux(p, sizeof(float) * npix * hp.n_chan);
    if (s != MOFF_OK) return s;
    moff::UvArgs u{};
    u.S = dL_dimage;
    u.Pn = p->d_Pn;
    u.out = static_cast<float*>(p->d_aux);
    u.N = hp.N;
    u.n_chan = hp.n_chan;
    u.a0 = hp.a0;
    u.scale = 1.0;
    if (moff::launch_uv_adjoint_shift(u, st) != hipSuccess) return MOFF_ERR_HIP;
    R = u.out;
  }
  moff::GradFinalArgs gf{};
  gf.R = R;
  gf.Pp = p->d_Pp;
  gf.gains = reinterpret_cast<const float2*>(gains);
  gf.ant_type = p->d_ant_type;
  gf.grad = reinterpret_cast<float2*>(dL_dgains);
  gf.N = hp.N;
  gf.n_ant = hp.n_ant;
  gf.n_chan = hp.n_chan;
  gf.n_types = hp.n_ktypes;
  gf.subtract = (hp.flags & (MOFF_AUTOCORR_NONE | MOFF_AUTOCORR_UV)) ? 0 : 1;
  gf.scale = 2.0 * image_scale(hp, n_time);

  const int av = std::min<int>(p->adj_variant, static_cast<int>(hp.variants.size()) - 1);
  const HostPlan::Variant& AV = hp.variants[av];
  const size_t lds = moff::fused_lds_bytes(hp.N, av, AV.n_weights(), hp.n_ant);
  if (!force_staged && p->d_adj_slots[av] && lds <= size_t(159) * 1024 &&
      moff::adjoint_fused_blocks_per_cu(hp.N, av, ci4, p->adj_waves, lds) > 0) {
    // fused: every frame's grid, field and adjoint stay in LDS
    const int per_slice = AV.shape.SX * hp.n_chan;
    const int resident =
        std::max(1, moff::adjoint_fused_blocks_per_cu(hp.N, av, ci4, p->adj_waves, lds)) * std::max(1, p->cu_count);
    const int slices = static_cast<int>(
        std::max<int64_t>(1, std::min<int64_t>({(2 * resident + per_slice - 1) / per_slice, n_time, 64})));
    const int parts = slices * AV.shape.SX;
    const size_t na = static_cast<size_t>(hp.n_chan) * hp.n_ant;
    const size_t d_bytes = (sizeof(double2) * na * (parts + 1) + sizeof(double) * na + 255) / 256 * 256;
    s = ensure_workspace(p, d_bytes + sizeof(float) * moff::fused_lane_values(hp.N, av) * hp.n_chan);
    if (s != MOFF_OK) return s;
    double2* Dp = static_cast<double2*>(p->d_ws);
    double2* D = Dp + na * parts;
    double* Q = reinterpret_cast<double*>(D + na);
    float* Rl = reinterpret_cast<float*>(static_cast<char*>(p->d_ws) + d_bytes);
    if (moff::launch_adjoint_sensitivity(R, hp.N, av, hp.n_chan, Rl, st) != hipSuccess) return MOFF_ERR_HIP;
    moff::AdjFusedArgs a{};
    a.E = E;
    a.gains = reinterpret_cast<const float2*>(gains);
    a.prog = p->d_prog[av];
    a.progw = p->d_progw[av];
    a.cell0 = p->d_cell0[av];
    a.prog_len = AV.prog_len;
    a.wave_rows = AV.wave_rows ? 1 : 0;
    a.dst_entries = AV.dst_entries ? 1 : 0;
    a.progress_prio = resident > std::max(1, p->cu_count) ? 1 : 0;
    a.weights = p->d_weights[av];
    a.n_weights = AV.n_weights();
    a.tw = p->d_tw;
    a.slots = p->d_adj_slots[av];
    a.Rl = Rl;
    a.n_ant = hp.n_ant;
    a.n_chan = hp.n_chan;
    a.n_taps = hp.n_taps;
    a.n_time = n_time;
    a.slices = slices;
    a.Dp = Dp;
    if (p->timing && hipEventRecord(p->ev0, st) != hipSuccess) return MOFF_ERR_HIP;
    if (moff::launch_adjoint_fused(a, hp.N, av, ci4, p->adj_waves, per_slice * slices, st) != hipSuccess)
      return MOFF_ERR_HIP;
    if (p->timing) {
      if (hipEventRecord(p->ev1, st) != hipSuccess) return MOFF_ERR_HIP;
      p->timed = true;
    }
    if (moff::launch_adjoint_reduce(Dp, parts, hp.n_chan, hp.n_ant, D, st) != hipSuccess) return MOFF_ERR_HIP;
    if (moff::launch_antenna_power(E, ci4, n_time, hp.n_chan, hp.n_ant, Q, st) != hipSuccess) return MOFF_ERR_HIP;
    gf.D = D;
    gf.Q = Q;
    return hip_status(moff::launch_grad_final(gf, st));
  }

  // staged: per time chunk, grids, fields and adjoint grids through HBM
  const size_t L2 = static_cast<size_t>(hp.L) * hp.L;
  const size_t gp_frame = static_cast<size_t>(V.shape.SX) * hp.L * V.NZR;
  const size_t d_bytes = sizeof(double) * 2 * hp.n_chan * hp.n_ant;
  const size_t q_bytes = sizeof(double) * hp.n_chan * hp.n_ant;
  // time chunk: the per-chunk grids, fields and adjoint grids within ~2 GiB
  const size_t per_t = sizeof(float2) * (L2 + npix + gp_frame) * hp.n_chan;
  int64_t chunk = std::max<int64_t>(1, static_cast<int64_t>((size_t(2) << 30) / per_t));
  chunk = std::min(chunk, n_time);
  const size_t eg_bytes = sizeof(float2) * L2 * hp.n_chan * chunk;
  const size_t y_bytes = sizeof(float2) * npix * hp.n_chan * chunk;
  const size_t gp_bytes = sizeof(float2) * gp_frame * hp.n_chan * chunk;
  s = ensure_workspace(p, d_bytes + q_bytes + eg_bytes + y_bytes + gp_bytes);
  if (s != MOFF_OK) return s;
  char* ws = static_cast<char*>(p->d_ws);
  double2* D = reinterpret_cast<double2*>(ws);
  double* Q = reinterpret_cast<double*>(ws + d_bytes);
  float2* Eg = reinterpret_cast<float2*>(ws + d_bytes + q_bytes);
  float2* Y = reinterpret_cast<float2*>(ws + d_bytes + q_bytes + eg_bytes);
  float2* Gp = reinterpret_cast<float2*>(ws + d_bytes + q_bytes + eg_bytes + y_bytes);
  if (moff::launch_zero(ws, d_bytes + q_bytes, st) != hipSuccess) return MOFF_ERR_HIP;
  const size_t sample_bytes = ci4 ? 1 : sizeof(float2);
  for (int64_t t0 = 0; t0 < n_time; t0 += chunk) {
    const int64_t nt = std::min(chunk, n_time - t0);
    const void* Ec = static_cast<const char*>(E) + static_cast<size_t>(t0) * hp.n_chan * hp.n_ant * sample_bytes;
    moff::GridArgs g = grid_args(p, Ec, nt, gains);
    g.Eg = Eg;
    hipError_t e = moff::launch_grid(g, ci4, st);
    moff::Fft2Args f{Eg, Y, p->d_tw};
    if (e == hipSuccess) e = moff::launch_fft2(f, hp.N, nt * hp.n_chan, st);
    moff::AdjFftArgs af{Y, R, Gp, p->d_tw, hp.n_chan};
    if (e == hipSuccess) e = moff::launch_adjoint_fft2(af, hp.N, nt * hp.n_chan, st);
    moff::DegridArgs dg{};
    dg.E = Ec;
    dg.Gp = Gp;
    dg.weights = p->d_weights[0];
    dg.ant_type = p->d_ant_type;
    dg.ant_cells = p->d_ant_cells;
    dg.ktype_k = p->d_ktype_k;
    dg.ktype_off = p->d_ktype_off;
    dg.D = D;
    dg.Q = Q;
    dg.n_ant = hp.n_ant;
    dg.n_chan = hp.n_chan;
    dg.n_taps = hp.n_taps;
    dg.SX = V.shape.SX;
    dg.L = hp.L;
    dg.M = V.M;
    dg.NZR = V.NZR;
    dg.NJ = V.NJ;
    dg.n_time = nt;
    if (e == hipSuccess) e = moff::launch_degrid(dg, ci4, st);
    if (e != hipSuccess) return MOFF_ERR_HIP;
  }
  gf.D = D;
  gf.Q = Q;
  return hip_status(moff::launch_grad_final(gf, st));
}

// Host plan, then the device tables.  On an error the caller frees whatever
// was uploaded (p->device is set once the device is current).
moff_status plan_create_body(const moff_geometry* geom, int hip_device, moff_plan p) {
  std::string why;
  moff_status st = moff::build_host_plan(geom, &p->hp, &why);
  if (st != MOFF_OK) return st;
  if (hip_device >= 0) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device >= count) return MOFF_ERR_INVALID_ARG;
    DeviceGuard guard(hip_device);
    if (!guard.ok()) return MOFF_ERR_HIP;
    p->device = hip_device;
    const HostPlan& hp = p->hp;
    std::vector<double> Pp(hp.Pp);
    moff_status s = MOFF_OK;
    auto up = [&](moff_status r) {
      if (s == MOFF_OK) s = r;
    };
    for (size_t v = 0; v < hp.variants.size(); ++v) {
      up(upload(&p->d_prog[v], hp.variants[v].prog4.data(), sizeof(uint32_t) * hp.variants[v].prog4.size()));
      up(upload(&p->d_cell0[v], hp.variants[v].cell0.data(), sizeof(int32_t) * hp.variants[v].cell0.size()));
      if (!hp.variants[v].progw.empty())
        up(upload(&p->d_progw[v], hp.variants[v].progw.data(), sizeof(float) * hp.variants[v].progw.size()));
      up(upload(&p->d_weights[v], hp.variants[v].weights.data(), sizeof(float) * hp.variants[v].weights.size()));
    }
    if (hp.mfma.prec) {
      up(upload(&p->d_mfma_prog, hp.mfma.prog.data(), sizeof(GatherEntry) * hp.mfma.prog.size()));
      up(upload(&p->d_mfma_dft, hp.mfma.dft.data(), sizeof(uint16_t) * hp.mfma.dft.size()));
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) p->cu_count = prop.multiProcessorCount;
    if (hip_device < kMaxDevices) {
      void* sp = nullptr;
      up(noalloc_scratch(hip_device, &sp));
    }
    up(upload(&p->d_tw, hp.twiddle.data(), sizeof(float) * hp.twiddle.size()));
    up(upload(&p->d_Pp, Pp.data(), sizeof(double) * Pp.size()));
    up(upload(&p->d_Pn, hp.Pn.data(), sizeof(double) * hp.Pn.size()));
    for (size_t v = 0; v < hp.variants.size(); ++v)
      if (!hp.variants[v].slots.empty())
        up(upload(&p->d_adj_slots[v], hp.variants[v].slots.data(), sizeof(uint32_t) * hp.variants[v].slots.size()));
    up(upload(&p->d_ant_type, hp.ant_ktype.data(), sizeof(int) * hp.ant_ktype.size()));
    up(upload(&p->d_ktab, hp.kvals.data(), sizeof(float) * hp.kvals.size()));
    up(upload(&p->d_csr_ptr, hp.csr_ptr.data(), sizeof(int) * hp.csr_ptr.size()));
    up(upload(&p->d_csr_ant, hp.csr_ant.data(), sizeof(int) * hp.csr_ant.size()));
    up(upload(&p->d_csr_tap, hp.csr_tap.data(), sizeof(int) * hp.csr_tap.size()));
    {
      std::vector<int> cells(2 * hp.n_ant);
      for (int a = 0; a < hp.n_ant; ++a) {
        cells[2 * a] = hp.ix0[a];
        cells[2 * a + 1] = hp.iy0[a];
      }
      up(upload(&p->d_ant_cells, cells.data(), sizeof(int) * cells.size()));
      up(upload(&p->d_ktype_k, hp.ktype_k.data(), sizeof(int) * hp.ktype_k.size()));
      up(upload(&p->d_ktype_off, hp.ktype_off.data(), sizeof(int) * hp.ktype_off.size()));
    }
    if (s != MOFF_OK) return s;
  }
  return MOFF_OK;
}

}  // namespace

extern "C" {

int moff_abi_version(void) { return MOFF_ABI_VERSION; }

const char* moff_status_str(moff_status s) {
  switch (s) {
    case MOFF_OK: return "ok";
    case MOFF_ERR_INVALID_ARG: return "invalid argument";
    case MOFF_ERR_GRID_NOT_POW2: return "grid_n must be a power of two in [8, 256]";
    case MOFF_ERR_FOOTPRINT_OVERFLOW: return "antenna footprints do not fit in the grid_n/2 aperture region";
    case MOFF_ERR_UNSUPPORTED: return "unsupported request";
    case MOFF_ERR_NOMEM: return "out of memory";
    case MOFF_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

moff_status moff_plan_create(const moff_geometry* geom, int hip_device, moff_plan* out) {
  if (!out) return MOFF_ERR_INVALID_ARG;
  *out = nullptr;
  moff_plan p = new (std::nothrow) moff_plan_s;
  if (!p) return MOFF_ERR_NOMEM;
  moff_status st;
  try {
    st = plan_create_body(geom, hip_device, p);
  } catch (...) {   // host containers of the plan build: a failed allocation
    st = MOFF_ERR_NOMEM;
  }
  if (st != MOFF_OK) {
    if (p->device >= 0) {
      DeviceGuard guard(p->device);
      free_device(p);
    }
    delete p;
    return st;
  }
  *out = p;
  return MOFF_OK;
}
moff_status moff_plan_destroy(moff_plan p) {
  if (!p) return MOFF_OK;
  if (p->device >= 0) {
    DeviceGuard guard(p->device);
    (void)hipDeviceSynchronize();
    free_device(p);
  }
  delete p;
  return MOFF_OK;
}

moff_status moff_plan_query(moff_plan p, int32_t* cells, double* cell_m, double* lm_per_pixel, int32_t* grid_n) {
  if (!p) return MOFF_ERR_INVALID_ARG;
  const HostPlan& hp = p->hp;
  if (cells)
    for (int a = 0; a < hp.n_ant; ++a) {
      cells[2 * a] = hp.ix0[a];
      cells[2 * a + 1] = hp.iy0[a];
    }
  if (cell_m) *cell_m = hp.cell_m;
  if (lm_per_pixel) std::copy(hp.lm_per_pixel.begin(), hp.lm_per_pixel.end(), lm_per_pixel);
  if (grid_n) *grid_n = hp.N;
  return MOFF_OK;
}

moff_status moff_plan_set_timing(moff_plan p, int enable) {
  if (!p) return MOFF_ERR_INVALID_ARG;
  if (p->device < 0) return MOFF_ERR_UNSUPPORTED;
  if (enable && !p->ev0) {
    DeviceGuard guard(p->device);
    if (!guard.ok()) return MOFF_ERR_HIP;
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess) return MOFF_ERR_HIP;
  }
  p->timing = enable != 0;
  p->timed = false;
  return MOFF_OK;
}

moff_status moff_plan_last_kernel_ms(moff_plan p, double* ms) {
  if (!p || !ms || !p->timing || !p->timed) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  if (hipEventSynchronize(p->ev1) != hipSuccess) return MOFF_ERR_HIP;
  float f = 0.f;
  if (hipEventElapsedTime(&f, p->ev0, p->ev1) != hipSuccess) return MOFF_ERR_HIP;
  *ms = f;
  return MOFF_OK;
}

moff_status moff_plan_power_pattern(moff_plan p, int32_t ktype, double* out) {
  if (!p || !out || ktype < 0 || ktype >= p->hp.n_ktypes) return MOFF_ERR_INVALID_ARG;
  const size_t n = static_cast<size_t>(p->hp.N) * p->hp.N;
  std::memcpy(out, p->hp.Pp.data() + n * ktype, n * sizeof(double));
  return MOFF_OK;
}

moff_status moff_plan_gather_program(moff_plan p, int32_t variant, int32_t w, uint32_t* out, float* weights,
                                     int32_t* prog_len, int32_t* n_threads, int32_t* n_classes, int32_t* row_pitch,
                                     int32_t* n_weights) {
  if (!p || variant < 0 || variant >= static_cast<int32_t>(p->hp.variants.size())) return MOFF_ERR_INVALID_ARG;
  const HostPlan::Variant& V = p->hp.variants[variant];
  if (prog_len) *prog_len = V.prog_len;
  if (n_threads) *n_threads = V.shape.NT;
  if (n_classes) *n_classes = V.shape.SX;
  if (row_pitch) *row_pitch = V.ZP;
  const int nw = V.n_weights();
  if (n_weights) *n_weights = nw;
  if (!out && !weights) return MOFF_OK;
  if (w < 0 || w >= V.shape.SX) return MOFF_ERR_INVALID_ARG;
  if (out) {
    const size_t n = static_cast<size_t>(V.prog_len) * V.shape.NT;
    const GatherEntry* src = V.prog.data() + n * w;
    for (size_t i = 0; i < n; ++i) {
      out[2 * i] = src[i].x;
      out[2 * i + 1] = src[i].y;
    }
  }
  if (weights) std::memcpy(weights, V.weights.data() + static_cast<size_t>(2) * nw * w, sizeof(float) * 2 * nw);
  return MOFF_OK;
}

moff_status moff_plan_mfma_tables(moff_plan p, uint32_t* prog, uint16_t* dft, int32_t* prog_len, int32_t* n_threads,
                                  int32_t* row_pitch, int32_t* grid_base, int32_t* dft_len) {
  if (!p) return MOFF_ERR_INVALID_ARG;
  const HostPlan::Mfma& T = p->hp.mfma;
  if (!T.prec) return MOFF_ERR_UNSUPPORTED;
  if (prog_len) *prog_len = T.prog_len;
  if (n_threads) *n_threads = T.NT;
  if (row_pitch) *row_pitch = T.pitch;
  if (grid_base) *grid_base = T.grid_base;
  if (dft_len) *dft_len = static_cast<int32_t>(T.dft.size());
  if (prog)
    for (size_t i = 0; i < T.prog.size(); ++i) {
      prog[2 * i] = T.prog[i].x;
      prog[2 * i + 1] = T.prog[i].y;
    }
  if (dft) std::memcpy(dft, T.dft.data(), sizeof(uint16_t) * T.dft.size());
  return MOFF_OK;
}

moff_status moff_plan_set_config(moff_plan p, int32_t variant, int32_t slices) {
  if (!p || variant < 0 || variant >= n_variants(p->hp) || slices < 0 || slices > 256) return MOFF_ERR_INVALID_ARG;
  p->variant = variant;
  p->adj_variant = variant;
  p->slices = slices;
  p->tuned = false;
  return MOFF_OK;
}

moff_status moff_plan_get_config(moff_plan p, int64_t n_time, int32_t* variant, int32_t* slices, int32_t* grid,
                                 int32_t* threads, int32_t* n_variants_out, int32_t* tuned) {
  if (!p || n_time < 1) return MOFF_ERR_INVALID_ARG;
  if (p->device < 0) return MOFF_ERR_UNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  const LaunchConfig lc = launch_config(p, n_time);
  if (variant) *variant = lc.variant;
  if (slices) *slices = lc.slices;
  if (grid) *grid = lc.grid;
  if (threads) *threads = footprint(p, lc.variant).threads;
  if (n_variants_out) *n_variants_out = n_variants(p->hp);
  if (tuned) *tuned = p->tuned ? 1 : 0;
  return MOFF_OK;
}

moff_status moff_plan_autotune(moff_plan p, const void* E, int64_t n_time, const float* gains, void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const HostPlan& hp = p->hp;
  const size_t img_bytes = sizeof(float) * static_cast<size_t>(hp.N) * hp.N * hp.n_chan;
  float* img = nullptr;
  if (hipMalloc(&img, img_bytes) != hipSuccess) return MOFF_ERR_NOMEM;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(img);
    return MOFF_ERR_HIP;
  }
  const int saved_v = p->variant, saved_s = p->slices;
  const bool saved_timing = p->timing;
  p->timing = false;
  float best = 1e30f;
  int bv = saved_v, bs = saved_s;
  // every timed candidate (at most 11 slice counts per shape variant)
  struct Timed {
    int v, sl;
    float ms;
  } timed[moff::kMaxVariants * 11];
  int n_timed = 0;
  moff_status result = MOFF_OK;
  {
    // Bring the device to its steady clocks first (about 200 ms of the default
    // launch): candidates are swept in order, and the first ones would
    // otherwise be timed on a device that is still ramping up.
    const LaunchConfig lc0 = launch_config(p, n_time);
    float spent = 0.f;
    for (int i = 0; i < 256 && spent < 200.f && result == MOFF_OK; ++i) {
      if (hipEventRecord(e0, st) != hipSuccess) result = MOFF_ERR_HIP;
      if (result == MOFF_OK) result = fused_run_cfg(p, lc0, E, n_time, gains, img, nullptr, true, st);
      if (result == MOFF_OK && hipEventRecord(e1, st) != hipSuccess) result = MOFF_ERR_HIP;
      if (result == MOFF_OK && hipEventSynchronize(e1) != hipSuccess) result = MOFF_ERR_HIP;
      float one = 0.f;
      if (result == MOFF_OK && hipEventElapsedTime(&one, e0, e1) != hipSuccess) result = MOFF_ERR_HIP;
      spent += one;
    }
  }
  for (int v = 0; v < n_variants(hp) && result == MOFF_OK; ++v) {
    const KernelFootprint f = footprint(p, v);
    if (f.lds > size_t(159) * 1024) continue;
    const int per_slice = f.per_slice, resident = f.resident;
    int cand[11], n_cand = 0;   // fixed size: the tuner allocates nothing on the host
    for (int k = 1; k <= 4; ++k) cand[n_cand++] = (k * resident + per_slice - 1) / per_slice;  // whole rounds
    for (int sl : {1, 2, 4, 8, 16, 32, 64}) cand[n_cand++] = sl;
    std::sort(cand, cand + n_cand);
    n_cand = static_cast<int>(std::unique(cand, cand + n_cand) - cand);
    for (int ci = 0; ci < n_cand; ++ci) {
      const int sl = cand[ci];
      if (sl < 1 || sl > 256 || sl > n_time || result != MOFF_OK) continue;
      {
        p->variant = v;
        p->slices = sl;
        const LaunchConfig lc = launch_config(p, n_time);
        result = fused_run_cfg(p, lc, E, n_time, gains, img, nullptr, true, st);   // warm-up
        if (result != MOFF_OK) break;
        // the fastest of several timed batches of back-to-back calls: candidates
        // are ranked by their steady-state time (as in use, call after call),
        // and near-equal ones by their undisturbed batch, not one noisy sample
        float ms = 1e30f;
        for (int rep = 0; rep < kTuneReps && result == MOFF_OK; ++rep) {
          if (hipEventRecord(e0, st) != hipSuccess) result = MOFF_ERR_HIP;
          for (int b = 0; b < kTuneBatch && result == MOFF_OK; ++b)
            result = fused_run_cfg(p, lc, E, n_time, gains, img, nullptr, true, st);
          if (result == MOFF_OK && hipEventRecord(e1, st) != hipSuccess) result = MOFF_ERR_HIP;
          if (result == MOFF_OK && hipEventSynchronize(e1) != hipSuccess) result = MOFF_ERR_HIP;
          float one = 0.f;
          if (result == MOFF_OK && hipEventElapsedTime(&one, e0, e1) != hipSuccess) result = MOFF_ERR_HIP;
          if (result == MOFF_OK) ms = std::min(ms, one);
        }
        if (result == MOFF_OK && n_timed < static_cast<int>(sizeof(timed) / sizeof(timed[0]))) {
          timed[n_timed++] = {v, sl, ms};
          best = std::min(best, ms);
        }
      }
    }
  }
  // Of the candidates within kTuneSlack of the fastest call, the one with the
  // fewest time slices (then the fastest): fewer per-slice partial images to
  // write and read back, and less scratch, at the same time per call.
  {
    float chosen = 1e30f;
    int chosen_sl = 1 << 30;
    for (int i = 0; i < n_timed; ++i) {
      const Timed& c = timed[i];
      if (c.ms > best * (1.f + kTuneSlack)) continue;
      if (c.sl < chosen_sl || (c.sl == chosen_sl && c.ms < chosen)) {
        chosen = c.ms;
        chosen_sl = c.sl;
        bv = c.v;
        bs = c.sl;
      }
    }
  }
  // The fused gain adjoint's register budget (moff_plan_set_adjoint_waves):
  // where more than one is built, time each on the same input with the tuned
  // forward image as the pixel sensitivities, and keep the fastest.  Not for
  // the reduced-precision plans, whose tuning is about their image path.
  int bw = p->adj_waves, bav = p->adj_variant;
  const int wmax = moff::adjoint_waves_max(hp.N);
  const bool ci4 = hp.flags & MOFF_IN_CI4;
  if (result == MOFF_OK && !is_mfma(hp)) {
    p->variant = bv;
    p->slices = bs;
    float* grad = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&grad), sizeof(float) * 2 * hp.n_chan * hp.n_ant) != hipSuccess)
      result = MOFF_ERR_NOMEM;
    float best_adj = 1e30f;
    for (int av = 0; av < n_variants(hp) && result == MOFF_OK; ++av) {
      const size_t alds = moff::fused_lds_bytes(hp.N, av, hp.variants[av].n_weights(), hp.n_ant);
      if (!p->d_adj_slots[av] || alds > size_t(159) * 1024) continue;
      for (int wv = 1; wv <= wmax && result == MOFF_OK; ++wv) {
        if (moff::adjoint_fused_blocks_per_cu(hp.N, av, ci4, wv, alds) <= 0) continue;
        p->adj_variant = av;
        p->adj_waves = wv;
        result = gain_vjp(p, E, n_time, gains, img, grad, st, false);   // warm-up (and workspace)
        float ms = 1e30f;
        for (int rep = 0; rep < 2 && result == MOFF_OK; ++rep) {
          if (hipEventRecord(e0, st) != hipSuccess) result = MOFF_ERR_HIP;
          if (result == MOFF_OK) result = gain_vjp(p, E, n_time, gains, img, grad, st, false);
          if (result == MOFF_OK && hipEventRecord(e1, st) != hipSuccess) result = MOFF_ERR_HIP;
          if (result == MOFF_OK && hipEventSynchronize(e1) != hipSuccess) result = MOFF_ERR_HIP;
          float one = 0.f;
          if (result == MOFF_OK && hipEventElapsedTime(&one, e0, e1) != hipSuccess) result = MOFF_ERR_HIP;
          if (result == MOFF_OK) ms = std::min(ms, one);
        }
        if (result == MOFF_OK && ms < best_adj) {
          best_adj = ms;
          bw = wv;
          bav = av;
        }
      }
    }
    (void)hipStreamSynchronize(st);
    if (grad) (void)hipFree(grad);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(img);
  p->timing = saved_timing;
  if (result != MOFF_OK) {
    p->variant = saved_v;
    p->slices = saved_s;
    p->adj_waves = 1;
    p->adj_variant = saved_v;
    return result;
  }
  p->variant = bv;
  p->slices = bs;
  p->adj_waves = bw;
  p->adj_variant = bav;
  p->tuned = true;
  return MOFF_OK;
}

moff_status moff_plan_set_adjoint_waves(moff_plan p, int32_t waves_per_simd) {
  if (!p) return MOFF_ERR_INVALID_ARG;
  if (waves_per_simd < 1) return MOFF_ERR_INVALID_ARG;
  if (waves_per_simd > moff::adjoint_waves_max(p->hp.N)) return MOFF_ERR_UNSUPPORTED;
  p->adj_waves = waves_per_simd;
  return MOFF_OK;
}

moff_status moff_plan_get_adjoint_waves(moff_plan p, int32_t* waves_per_simd, int32_t* max_waves_per_simd) {
  if (!p) return MOFF_ERR_INVALID_ARG;
  if (waves_per_simd) *waves_per_simd = p->adj_waves;
  if (max_waves_per_simd) *max_waves_per_simd = moff::adjoint_waves_max(p->hp.N);
  return MOFF_OK;
}

moff_status moff_image(moff_plan p, const void* E, int64_t n_time, const float* gains, float* image,
                       void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !image || !aligned16(image) || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!uv_rule(p->hp)) return fused_run(p, E, n_time, gains, image, nullptr, true, st);
  // uv-plane rule: accumulate S (and A) first, then remove the zero-spacing component
  const HostPlan& hp = p->hp;
  const size_t s_bytes = sizeof(float) * static_cast<size_t>(hp.N) * hp.N * hp.n_chan;
  const size_t a_bytes = sizeof(double) * hp.n_chan * hp.n_ktypes;
  s = ensure_aux(p, s_bytes + a_bytes);
  if (s != MOFF_OK) return s;
  float* S = static_cast<float*>(p->d_aux);
  double* A = reinterpret_cast<double*>(static_cast<char*>(p->d_aux) + s_bytes);
  if (moff::launch_zero(p->d_aux, s_bytes + a_bytes, st) != hipSuccess) return MOFF_ERR_HIP;
  s = fused_run(p, E, n_time, gains, S, A, false, st);
  if (s != MOFF_OK) return s;
  return uv_finalize(p, S, n_time, image, st);
}

moff_status moff_image_noalloc(moff_plan p, const void* E, int64_t n_time, const float* gains, float* image,
                               void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !image || !aligned16(image) || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  const HostPlan& hp = p->hp;
  if (uv_rule(hp)) return MOFF_ERR_UNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (p->device < kMaxDevices) ptr = g_scratch_ptr[p->device];
  }
  if (!ptr) return MOFF_ERR_UNSUPPORTED;   // set at plan creation; absent only beyond kMaxDevices
  // The plan's launch configuration, with fewer time slices while its scratch
  // would not fit (results differ only in float32 rounding order).
  LaunchConfig lc = launch_config(p, n_time);
  while (lc.slices > 1 && fused_scratch(hp, lc, n_time).total() > MOFF_NOALLOC_SCRATCH_BYTES) {
    --lc.slices;
    lc.grid = launch_grid(hp, lc.variant, lc.slices);
  }
  if (fused_scratch(hp, lc, n_time).total() > MOFF_NOALLOC_SCRATCH_BYTES) return MOFF_ERR_UNSUPPORTED;
  return fused_run_cfg(p, lc, E, n_time, gains, image, nullptr, true, static_cast<hipStream_t>(stream), ptr);
}

moff_status moff_accumulate(moff_plan p, const void* E, int64_t n_time, const float* gains, float* S, double* A,
                            void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !S || !A || !aligned16(S) || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  return fused_run(p, E, n_time, gains, S, A, false, static_cast<hipStream_t>(stream));
}

moff_status moff_finalize(moff_plan p, const float* S, const double* A, int64_t n_time_total, float* image,
                          void* stream) {
  // Only scales and subtracts per pixel: no per-sample indexing, so no limit on
  // n_time_total beyond being a positive count.
  if (!p) return MOFF_ERR_INVALID_ARG;
  if (p->device < 0) return MOFF_ERR_UNSUPPORTED;
  if (n_time_total < 1 || !S || !A || !image || !aligned16(S) || !aligned16(image)) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  const HostPlan& hp = p->hp;
  if (uv_rule(hp)) return uv_finalize(p, S, n_time_total, image, static_cast<hipStream_t>(stream));
  moff::FinalizeArgs f{};
  f.S = S;
  f.A = A;
  f.Pp = p->d_Pp;
  f.out = image;
  f.N = hp.N;
  f.n_chan = hp.n_chan;
  f.n_types = hp.n_ktypes;
  f.subtract = (hp.flags & MOFF_AUTOCORR_NONE) ? 0 : 1;
  f.scale = image_scale(hp, n_time_total);
  return hip_status(moff::launch_finalize(f, static_cast<hipStream_t>(stream)));
}

moff_status moff_grid(moff_plan p, const void* E, int64_t n_time, const float* gains, float* eg, void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !eg || !aligned16(eg) || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  moff::GridArgs g = grid_args(p, E, n_time, gains);
  g.Eg = reinterpret_cast<float2*>(eg);
  return hip_status(moff::launch_grid(g, p->hp.flags & MOFF_IN_CI4, static_cast<hipStream_t>(stream)));
}

moff_status moff_self_power(moff_plan p, const void* E, int64_t n_time, const float* gains, double* A,
                            void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !A || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  moff::GridArgs g = grid_args(p, E, n_time, gains);
  g.A = A;
  return hip_status(moff::launch_self_power(g, p->hp.flags & MOFF_IN_CI4, static_cast<hipStream_t>(stream)));
}

moff_status moff_fft2(moff_plan p, const float* eg, int64_t n_frames, float* y, void* stream) {
  if (!p) return MOFF_ERR_INVALID_ARG;
  if (p->device < 0) return MOFF_ERR_UNSUPPORTED;
  if (n_frames < 1 || !eg || !y || !aligned16(eg) || !aligned16(y)) return MOFF_ERR_INVALID_ARG;
  if (n_frames * p->hp.variants[0].shape.SX >= (int64_t(1) << 31)) return MOFF_ERR_UNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  moff::Fft2Args f{reinterpret_cast<const float2*>(eg), reinterpret_cast<float2*>(y), p->d_tw};
  return hip_status(moff::launch_fft2(f, p->hp.N, n_frames, static_cast<hipStream_t>(stream)));
}

moff_status moff_detect_accumulate(moff_plan p, const float* y, int64_t n_time, float* S, void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!y || !S || !aligned16(y)) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  moff::DetectArgs d{reinterpret_cast<const float2*>(y), S, p->hp.N, p->hp.n_chan, n_time};
  return hip_status(moff::launch_detect(d, static_cast<hipStream_t>(stream)));
}

moff_status moff_image_staged(moff_plan p, const void* E, int64_t n_time, const float* gains, float* image,
                              void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !image || !aligned16(image) || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  const HostPlan& hp = p->hp;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool ci4 = hp.flags & MOFF_IN_CI4;
  const size_t npix = static_cast<size_t>(hp.N) * hp.N;
  const size_t s_bytes = sizeof(float) * npix * hp.n_chan;
  const size_t a_bytes = sizeof(double) * hp.n_chan * hp.n_ktypes;
  // time chunk: keep the per-chunk grids and fields within ~2 GiB
  const size_t per_t = (sizeof(float2) * (static_cast<size_t>(hp.L) * hp.L + npix)) * hp.n_chan;
  int64_t chunk = std::max<int64_t>(1, static_cast<int64_t>((size_t(2) << 30) / per_t));
  chunk = std::min(chunk, n_time);
  const size_t eg_bytes = sizeof(float2) * static_cast<size_t>(hp.L) * hp.L * hp.n_chan * chunk;
  const size_t y_bytes = sizeof(float2) * npix * hp.n_chan * chunk;
  s = ensure_workspace(p, s_bytes + a_bytes + eg_bytes + y_bytes);
  if (s != MOFF_OK) return s;
  char* ws = static_cast<char*>(p->d_ws);
  float* S = reinterpret_cast<float*>(ws);
  double* A = reinterpret_cast<double*>(ws + s_bytes);
  float2* Eg = reinterpret_cast<float2*>(ws + s_bytes + a_bytes);
  float2* Y = reinterpret_cast<float2*>(ws + s_bytes + a_bytes + eg_bytes);
  if (moff::launch_zero(ws, s_bytes + a_bytes, st) != hipSuccess) return MOFF_ERR_HIP;
  const size_t sample_bytes = ci4 ? 1 : sizeof(float2);
  for (int64_t t0 = 0; t0 < n_time; t0 += chunk) {
    const int64_t nt = std::min(chunk, n_time - t0);
    const void* Ec = static_cast<const char*>(E) + static_cast<size_t>(t0) * hp.n_chan * hp.n_ant * sample_bytes;
    moff::GridArgs g = grid_args(p, Ec, nt, gains);
    g.Eg = Eg;
    g.A = A;
    hipError_t e = moff::launch_grid(g, ci4, st);
    if (e == hipSuccess) e = moff::launch_self_power(g, ci4, st);
    moff::Fft2Args f{Eg, Y, p->d_tw};
    if (e == hipSuccess) e = moff::launch_fft2(f, hp.N, nt * hp.n_chan, st);
    moff::DetectArgs d{Y, S, hp.N, hp.n_chan, nt};
    if (e == hipSuccess) e = moff::launch_detect(d, st);
    if (e != hipSuccess) return MOFF_ERR_HIP;
  }
  if (uv_rule(hp)) return uv_finalize(p, S, n_time, image, st);
  moff::FinalizeArgs fa{};
  fa.S = S;
  fa.A = A;
  fa.Pp = p->d_Pp;
  fa.out = image;
  fa.N = hp.N;
  fa.n_chan = hp.n_chan;
  fa.n_types = hp.n_ktypes;
  fa.subtract = (hp.flags & MOFF_AUTOCORR_NONE) ? 0 : 1;
  fa.scale = image_scale(hp, n_time);
  return hip_status(moff::launch_finalize(fa, st));
}

moff_status moff_image_fx(moff_plan p, const void* E, int64_t n_time, const float* gains, float* image,
                          void* stream) {
  moff_status s = check_compute(p, n_time);
  if (s != MOFF_OK) return s;
  if (!E || !image || !aligned16(image) || (gains && !aligned16(gains))) return MOFF_ERR_INVALID_ARG;
  const HostPlan& hp = p->hp;
  // 4+4-bit samples are correlated in int32: |sum_t x_a x_b| <= 64 n_time
  if ((hp.flags & MOFF_IN_CI4) && n_time > (int64_t(1) << 24)) return MOFF_ERR_UNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok()) return MOFF_ERR_HIP;
  const bool keep_autos = (hp.flags & MOFF_AUTOCORR_NONE) != 0;
  if (!p->d_fx_ptr) {
    moff::FxTables t;
    try {
      moff::build_fx_tables(hp, keep_autos, &t);
    } catch (...) {   // the tables' host vectors: a failed allocation
      return MOFF_ERR_NOMEM;
    }
    moff_status u = upload(&p->d_fx_ptr, t.ptr.data(), sizeof(int32_t) * t.ptr.size());
    if (u == MOFF_OK) u = upload(&p->d_fx_ab, t.ab.data(), sizeof(int32_t) * t.ab.size());
    if (u == MOFF_OK) u = upload(&p->d_fx_x, t.xcorr.data(), sizeof(float) * t.xcorr.size());
    if (u != MOFF_OK) {
      for (void** q : {reinterpret_cast<void**>(&p->d_fx_ptr), reinterpret_cast<void**>(&p->d_fx_ab),
                       reinterpret_cast<void**>(&p->d_fx_x)})
        if (*q) {
          (void)hipFree(*q);
          *q = nullptr;
        }
      return u;
    }
    p->fx_NL = t.NL;
    p->fx_xs = t.xs;
  }
  const int NL = p->fx_NL, NTP = hp.n_ktypes * hp.n_ktypes;
  // workspace per channel; channels run in chunks that keep it within ~2 GiB
  const size_t v_per = sizeof(float2) * hp.n_ant * hp.n_ant;
  const size_t h_per = sizeof(float2) * NTP * NL * NL;
  const size_t r_per = sizeof(float2) * NL * NL;
  const size_t z_per = sizeof(float2) * NL * hp.N;
  const size_t per_chan = v_per + h_per + r_per + z_per;
  const int chunk = static_cast<int>(std::max<size_t>(
      1, std::min<size_t>({static_cast<size_t>(hp.n_chan), (size_t(2) << 30) / per_chan, size_t(65535)})));
  s = ensure_workspace(p, per_chan * chunk);
  if (s != MOFF_OK) return s;
  char* ws = static_cast<char*>(p->d_ws);
  moff::FxArgs a{};
  a.E = E;
  a.gains = reinterpret_cast<const float2*>(gains);
  a.n_ant = hp.n_ant;
  a.n_chan = hp.n_chan;
  a.n_types = hp.n_ktypes;
  a.n_time = n_time;
  a.N = hp.N;
  a.L = hp.L;
  a.NL = NL;
  a.xs = p->fx_xs;
  a.pair_ptr = p->d_fx_ptr;
  a.pair_ab = p->d_fx_ab;
  a.ktype_k = p->d_ktype_k;
  a.xcorr = p->d_fx_x;
  a.tw = p->d_tw;
  a.V = reinterpret_cast<float2*>(ws);
  a.H = reinterpret_cast<float2*>(ws + v_per * chunk);
  a.R = reinterpret_cast<float2*>(ws + (v_per + h_per) * chunk);
  a.Z = reinterpret_cast<float2*>(ws + (v_per + h_per + r_per) * chunk);
  a.out = image;
  a.scale = image_scale(hp, n_time);
  const bool ci4 = hp.flags & MOFF_IN_CI4;
  for (int c0 = 0; c0 < hp.n_chan; c0 += chunk) {
    a.c0 = c0;
    a.n_launch = std::min(chunk, hp.n_chan - c0);
    if (moff::launch_fx(a, ci4, static_cast<hipStream_t>(stream)) != hipSuccess) return MOFF_ERR_HIP;
  }
  return MOFF_OK;
}

moff_status moff_gain_vjp(moff_plan p, const void* E, int64_t n_time, const float* gains, const float* dL_dimage,
                          float* dL_dgains, void* stream) {
  return gain_vjp(p, E, n_time, gains, dL_dimage, dL_dgains, stream, false);
}

moff_status moff_gain_vjp_staged(moff_plan p, const void* E, int64_t n_time, const float* gains,
                                 const float* dL_dimage, float* dL_dgains, void* stream) {
  return gain_vjp(p, E, n_time, gains, dL_dimage, dL_dgains, stream, true);
}

}  // extern "C"
