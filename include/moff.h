/*
 * moff.h -- C ABI of the MI355X MOFF direct-imaging library.
 *
 * The Modular Optimal Frequency Fourier (MOFF) imager forms, for every time
 * sample t and frequency channel c (one "frame"), the image-plane field of the
 * calibrated, gridded antenna E-fields, squares it and averages it over time
 * (Thyagarajan et al., Sec. 2, MOFF imaging equation, eq. dirty-image-MOFF):
 *
 *   e[t,c,a]   = g[c,a] * E[t,c,a]                     calibration (Sec. 3)
 *   Eg[t,c]    = sum_a K_{p(a)} placed at (iy0_a,ix0_a) * e[t,c,a]
 *                                                      gridding (Sec. 3, E(r) = M E(a))
 *   Y[t,c]     = 2-D DFT of Eg zero-padded from N/2 x N/2 to N x N
 *                (exponent +2 pi i, unnormalised, pixel N/2 = phase centre)
 *                                                      spatial transform (Sec. 3)
 *   S[c]       = sum_t |Y[t,c]|^2                      squaring + time average (Sec. 3)
 *   A[c,p]     = sum_t sum_{a of type p} |e[t,c,a]|^2
 *   P_p        = |DFT of K_p|^2                        antenna power response (Sec. 4.2)
 *   I[c]       = (S[c] - sum_p A[c,p] P_p) / T         self-power removal (Sec. 4.2)
 *
 * Image pixel (r, q) of channel c is direction m = (r - N/2) lambda_c / (N cell),
 * l = (q - N/2) lambda_c / (N cell): rows follow y/m, columns follow x/l.
 *
 * Conventions for every call:
 *   - Geometry arrays are HOST pointers, copied at plan creation.
 *   - Data pointers (E, gains, grids, images, accumulators) are DEVICE pointers
 *     on the plan's device, owned by the caller, at least 16-byte aligned.
 *   - Calls enqueue work on `hip_stream` (a hipStream_t, NULL = default stream)
 *     and return without synchronising; argument validation is synchronous.
 *   - A plan's tables are fixed at creation; its only mutable state is the
 *     launch configuration (moff_plan_autotune / moff_plan_set_config /
 *     moff_plan_set_adjoint_waves), the timing switch and a device workspace,
 *     so concurrent calls must use different plans.
 *   - The workspace grows on demand: a call that needs more than the plan holds
 *     synchronises the device and allocates.  Under stream (graph) capture, make
 *     one eager call of the same shape first; captured calls then allocate
 *     nothing and record no memset nodes (buffers are cleared by a kernel).
 *   - On any error status the contents of output buffers are unspecified.
 *   - No C++ exception crosses this interface: a failed host allocation while
 *     a plan or its tables are built returns MOFF_ERR_NOMEM.
 *   - NaN / Inf inputs propagate; they are not checked.
 */
#ifndef MOFF_H
#define MOFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOFF_ABI_VERSION 1

typedef struct moff_plan_s* moff_plan;

typedef enum {
  MOFF_OK = 0,
  MOFF_ERR_INVALID_ARG = 1,         /* null pointer, non-positive size, bad flag, bad kernel table */
  MOFF_ERR_GRID_NOT_POW2 = 2,       /* grid_n not a power of two in [8, 256] */
  MOFF_ERR_FOOTPRINT_OVERFLOW = 3,  /* footprints do not fit in the grid_n/2 aperture region */
  MOFF_ERR_UNSUPPORTED = 4,         /* valid request the library does not implement (sizes, host-only plan) */
  MOFF_ERR_NOMEM = 5,               /* host or device allocation failed */
  MOFF_ERR_HIP = 6                  /* a HIP runtime call or kernel launch failed */
} moff_status;

/* geometry.flags bits */
enum {
  MOFF_IN_C64 = 0,         /* E is complex64: interleaved float32 (re, im) */
  MOFF_IN_CI4 = 1,         /* E is one byte per sample: re = high nibble, im = low nibble,
                              two's complement in [-8, 7] */
  MOFF_AUTOCORR_NONE = 2,  /* keep the antenna self power: I = S / T */
  MOFF_NORM_PAIRS = 4,     /* multiply the image by 1 / (n_ant (n_ant - 1)) (Sec. 5,
                              eq. wt-dirty-image-EPIC: average over antenna pairs) */
  MOFF_MFMA_F16 = 8,       /* reduced precision: the gridded field is rounded to IEEE
                              binary16 and the padded 2-D DFT (Sec. 3) runs as two dense
                              complex matrix products on the matrix cores with float32
                              accumulation; phase factors are made in float64 and rounded
                              once.  grid_n must be 64 or 128.  binary16 holds gridded
                              values up to 65504 in magnitude; components below 2^-14
                              lose relative precision.  Error against the exact image:
                              of order 2^-11 relative to the image peak (stated bound
                              16 * 2^-11 on max|dI| / max(S/T)).  The kernel keeps two
                              buffers of samples, grid and row-stage output in LDS, so
                              at grid_n 128 it takes about 1490 antennas (fewer with
                              large tables); beyond that, or when the sample and tap
                              offsets exceed 16 bits, plan creation returns
                              MOFF_ERR_UNSUPPORTED. */
  MOFF_MFMA_BF16 = 16,     /* as MOFF_MFMA_F16 with bfloat16 (float32 range, 8-bit
                              significand; stated bound 16 * 2^-8). At most one of the
                              two MFMA flags may be set. */
  MOFF_AUTOCORR_UV = 32    /* remove the autocorrelations with the uv-plane rule of
                              Sec. 4.2 instead of per-antenna subtraction: the
                              time-averaged image S / T is taken to the uv plane, the
                              tables' autocorrelation kernel a = sum_p n_p (K_p corr K_p)
                              (n_p antennas of type p) is subtracted at zero spacing,
                              scaled so the result is zero there, and the result is
                              transformed back: I = (S - beta sum_p n_p P_p) / T with
                              beta = sum_pix S / (N^2 a[0]).  Exact when footprints never
                              overlap and antennas have equal power; otherwise
                              cross-correlations of overlapping footprints at zero
                              spacing are removed too.  Not with MOFF_AUTOCORR_NONE. */
};

/*
 * Problem statement (Sec. 3, antenna-to-grid mapping): antenna positions and
 * illumination kernels, channel frequencies and the grid size.
 *
 *   n_ant, ant_xy_m : antenna positions, host float64 [n_ant][2] in metres,
 *                     (x, y); 2 <= n_ant <= 4000.
 *   n_ktypes, ktype_k, ktype_vals :
 *                     illumination tables, one per antenna type; type p is a
 *                     square ktype_k[p] x ktype_k[p] complex table (1 <= k <= 15),
 *                     row index u along y, column index v along x. ktype_vals
 *                     holds all tables back to back as interleaved float32
 *                     (re, im), row-major. 1 <= n_ktypes <= 4.
 *   ant_ktype       : host int32 [n_ant], type of each antenna.
 *   n_chan, freq_hz : channel centre frequencies, host float64 [n_chan] (> 0).
 *                     They set the pixel scale and the default cell size only;
 *                     footprints are channel-independent cells.
 *   grid_n          : FFT side N after two-fold zero padding; a power of two in
 *                     [8, 256]. Footprints must fit in the N/2 x N/2 aperture region.
 *   cell_m          : grid spacing in metres; 0 selects the default: half the
 *                     shortest wavelength, widened if needed so that the layout
 *                     span plus the widest footprint and one cell of slack fits
 *                     in N/2 cells.
 *   flags           : MOFF_IN_* | MOFF_AUTOCORR_NONE or MOFF_AUTOCORR_UV |
 *                     MOFF_NORM_PAIRS | MOFF_MFMA_F16 or MOFF_MFMA_BF16.
 *
 * Footprint placement: antenna a with a k x k table covers cells
 * ix0_a .. ix0_a + k - 1 with ix0_a = floor(x_a / cell - (k - 1) / 2 + 0.5)
 * (nearest cell, ties round up), the same for y; indices are then shifted so
 * the smallest ix0 and the smallest iy0 are 0.
 */
typedef struct {
  int32_t n_ant;
  const double* ant_xy_m;
  int32_t n_ktypes;
  const int32_t* ktype_k;
  const float* ktype_vals;
  const int32_t* ant_ktype;
  int32_t n_chan;
  const double* freq_hz;
  int32_t grid_n;
  double cell_m;
  uint32_t flags;
} moff_geometry;

/* ABI version of the loaded library (MOFF_ABI_VERSION at build time). */
int moff_abi_version(void);

/* Static, NUL-terminated description of a status code. Never NULL. */
const char* moff_status_str(moff_status s);

/*
 * Build a plan: the footprint cells (FP64 arithmetic), the gather tables keyed
 * by grid cell, the power patterns P_p (FP64 direct DFT, rounded to float32)
 * and the transform twiddles, computed once (Sec. 3: the mapping "must only be
 * determined once").  hip_device >= 0 uploads the tables to that device;
 * hip_device < 0 builds a host-only plan for moff_plan_query /
 * moff_plan_power_pattern (compute calls on it return MOFF_ERR_UNSUPPORTED).
 * *out receives the plan on MOFF_OK and NULL otherwise.
 */
moff_status moff_plan_create(const moff_geometry* geom, int hip_device, moff_plan* out);

/* Release a plan and its device memory. NULL is accepted. Synchronises the device. */
moff_status moff_plan_destroy(moff_plan plan);

/*
 * Host copies of the plan's placement results (Sec. 3, antenna-to-grid
 * mapping: each antenna's footprint is placed at its nearest grid cells, once
 * per geometry).  Any output may be NULL.
 *   cells        : int32 [n_ant][2] = (ix0_a, iy0_a) lower-left footprint cell,
 *                  by the placement rule stated with moff_geometry
 *   cell_m       : grid spacing used, metres
 *   lm_per_pixel : float64 [n_chan], direction-cosine step lambda_c / (N cell)
 *                  of the zero-padded transform (Sec. 3, spatial transform)
 *   grid_n       : N
 * Valid on host-only plans too.  Errors: MOFF_ERR_INVALID_ARG for a NULL plan.
 */
moff_status moff_plan_query(moff_plan plan, int32_t* cells, double* cell_m,
                            double* lm_per_pixel, int32_t* grid_n);

/*
 * Host copy of the float64 power pattern P_p of kernel type `ktype`
 * (Sec. 4.2, the antenna power response), out = float64 [N][N] in image pixel
 * order.
 */
moff_status moff_plan_power_pattern(moff_plan plan, int32_t ktype, double* out);

/*
 * Diagnostic copy of the fused kernel's cell-keyed gather program of shape
 * variant `variant` for output column class `w` (0 <= w < *n_classes).  Call with out = NULL to get the
 * sizes.  out receives uint32 [prog_len][n_threads][2] entries (x, y):
 *   x bits 0..11 antenna slot (n_ant = the zero slot), bits 12..22 weight
 *   index, bit 31 "cell complete: store"; y = LDS element iy * (*row_pitch) + n'
 *   of the folded-grid cell (iy, n').
 * weights (may be NULL) receives complex64 [n_weights] for class w:
 *   K[tap] * exp(+2 pi i j w / n_classes) at index j * n_taps + tap.
 * Used by host-side tests; the data never changes after plan creation.
 */
moff_status moff_plan_gather_program(moff_plan plan, int32_t variant, int32_t w, uint32_t* out, float* weights,
                                     int32_t* prog_len, int32_t* n_threads, int32_t* n_classes,
                                     int32_t* row_pitch, int32_t* n_weights);

/*
 * Tables of the reduced-precision (MOFF_MFMA_*) path, for host-side tests.
 * Sizes first (any pointer may be NULL): prog_len entries per lane,
 * n_threads gather lanes (the lanes of the kernel's gather waves; its matrix
 * waves come on top), row_pitch 16-bit elements per grid row, grid_base the
 * LDS byte offset of the first of the two 16-bit aperture grids, dft_len
 * 16-bit words of phase-factor operands.
 *   prog : uint32 [prog_len][n_threads][2] gather entries (x, y) over the
 *          non-empty aperture cells (iy, ix), in LDS byte offsets into the
 *          first sample buffer and grid: x low half = 8 * antenna
 *          (8 * n_ant is an all-zero slot), x high half =
 *          16 * (n_ant + 1) + 8 * tap (kernel taps of all types back to back,
 *          after two buffers of n_ant + 1 samples);
 *          y = 0, or on the last entry of a cell y = grid_base +
 *          2 * (iy * row_pitch + ix), where the cell's real part is stored (its
 *          imaginary part is grid_n / 2 elements further on).
 *   dft  : uint16 [2][grid_n / 64][2][grid_n / 64][2][64][8] binary16 or
 *          bfloat16 bit patterns, indexed
 *          [stage][base block][half][k-step][part][lane][slot], for the base
 *          half (index n < grid_n / 2) of each transform; the other half
 *          follows by conjugation (column grid_n - n of the row transform is
 *          the conjugate of column n, and likewise for rows of the column
 *          transform).  Stage 0 = row transform exp(+2 pi i ix (q - N/2) / N) /
 *          (N/2) at column q = 32 block + 16 half + lane % 16 and
 *          ix = 32 k-step + 8 (lane / 16) + slot; stage 1 = column transform
 *          exp(+2 pi i iy (r - N/2) / N) at row r = 32 block + 16 half +
 *          lane % 16 and iy likewise.  Part 0 holds the real part, part 1 the
 *          imaginary part, except at n = 0, where part 0 holds the (real) phase
 *          vector of n - N/2 = -N/2 and part 1 that of n - N/2 = 0 (all ones),
 *          each with the stage's scale.
 * MOFF_ERR_UNSUPPORTED if the plan has no MFMA flag.
 */
moff_status moff_plan_mfma_tables(moff_plan plan, uint32_t* prog, uint16_t* dft, int32_t* prog_len,
                                  int32_t* n_threads, int32_t* row_pitch, int32_t* grid_base, int32_t* dft_len);

/*
 * Launch configuration of the fused path.  The frame transform has one or two
 * shape variants per grid size (how output columns are split across
 * workgroups, threads per workgroup); a launch also chooses the number of time
 * slices: each (column class, channel, slice) is one workgroup, and per-slice
 * partial sums are reduced afterwards in a fixed order.
 *
 * moff_plan_autotune times every candidate (variant x slices, including the
 * slice counts that fill whole rounds of resident workgroups) with HIP events
 * on `hip_stream` using the caller's data and synchronises the stream.  It
 * first runs the default shape for about 200 ms so that no candidate is timed
 * on a cold device, then takes each candidate's time as the best of three
 * batches of three back-to-back calls, and keeps, of the candidates within 3 %
 * of the fastest, the one with the fewest time slices (less scratch and fewer
 * partial images to reduce).  Later results do not depend on the choice
 * beyond float32 rounding order.  Unless the plan has a MOFF_MFMA_* flag, it also times the
 * fused gain adjoint (moff_gain_vjp) for every shape variant and register
 * budget it is built with (see moff_plan_set_adjoint_waves), on the same
 * samples and gains with the tuned image as the pixel sensitivities, and
 * keeps the fastest.  moff_plan_set_config forces a choice (slices = 0:
 * heuristic) and gives the adjoint the same shape variant; moff_plan_get_config
 * reports the configuration a call with n_time samples would use.  Any output
 * of get_config may be NULL.
 */
moff_status moff_plan_autotune(moff_plan plan, const void* E_dev, int64_t n_time, const float* gains_dev,
                               void* hip_stream);

/*
 * Register budget of the fused gain adjoint (moff_gain_vjp): the least number
 * of waves per SIMD its registers are sized for (1, the default: as many as the
 * kernel wants).  The adjoint reads its pixel sensitivities and its antennas'
 * descriptors from memory as each frame needs them, so at every grid size it
 * fits two waves per SIMD without spilling; at grid_n 128 a budget of 3 runs
 * three waves (the smaller shape variant without spilling).  Which is fastest
 * depends on the workload; results are the same either way.
 * max_waves_per_simd = 3 at grid_n 128, 2 at 256, 1 otherwise;
 * set_adjoint_waves returns MOFF_ERR_UNSUPPORTED above it and
 * MOFF_ERR_INVALID_ARG below 1.  Outputs of get_adjoint_waves may be NULL.
 */
moff_status moff_plan_set_adjoint_waves(moff_plan plan, int32_t waves_per_simd);
moff_status moff_plan_get_adjoint_waves(moff_plan plan, int32_t* waves_per_simd, int32_t* max_waves_per_simd);
moff_status moff_plan_set_config(moff_plan plan, int32_t variant, int32_t slices);
moff_status moff_plan_get_config(moff_plan plan, int64_t n_time, int32_t* variant, int32_t* slices, int32_t* grid,
                                 int32_t* threads, int32_t* n_variants, int32_t* tuned);

/*
 * Kernel timing.  With timing enabled, every fused call records a pair of HIP
 * events on its stream around the fused kernel (not the small reduction that
 * may follow it).  moff_plan_last_kernel_ms waits for the most recent fused
 * call and returns that kernel's duration in milliseconds (MOFF_ERR_INVALID_ARG
 * if timing is off or no fused call has been made since it was turned on).
 */
moff_status moff_plan_set_timing(moff_plan plan, int enable);
moff_status moff_plan_last_kernel_ms(moff_plan plan, double* ms);

/* ---------------------------------------------------------------------------
 * Fused path: one kernel per call runs ingest, calibration, gridding, the
 * padded 2-D FFT, squaring and accumulation for all frames; the image is
 * produced without any per-frame HBM round trip.
 * ------------------------------------------------------------------------- */

/*
 * Time-averaged image with self power removed (or kept, MOFF_AUTOCORR_NONE).
 *   E_dev     : [n_time][n_chan][n_ant] samples in the plan's input format
 *   n_time    : number of time samples T >= 1 (the integration)
 *   gains_dev : complex64 [n_chan][n_ant] calibration gains g, or NULL for g = 1;
 *               a zero gain flags the antenna (App. A: flags are weights)
 *   image_dev : float32 [n_chan][N][N], overwritten with I
 */
moff_status moff_image(moff_plan plan, const void* E_dev, int64_t n_time,
                       const float* gains_dev, float* image_dev, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): moff_image
 * with no allocation.  Same arguments, output and errors as moff_image; the
 * result equals moff_image's up to float32 rounding order (bitwise when both
 * use the same launch configuration).  Its scratch -- the per-slice partial
 * sums and float64 running sums of the fused call -- lives in one fixed
 * MOFF_NOALLOC_SCRATCH_BYTES device array per GPU, taken when the first plan
 * on that GPU is created and held until the process ends; the call makes no
 * hipMalloc, hipFree or other allocating call.  The plan's launch
 * configuration is used with fewer time slices when its scratch would not fit.
 * Every call on one GPU (from any plan) shares that array and overwrites it
 * without clearing (nothing in it needs to start at zero), so calls that
 * overlap on one GPU race: serialise them on one stream.
 * Errors as moff_image, plus MOFF_ERR_UNSUPPORTED when even one time slice
 * needs more scratch than MOFF_NOALLOC_SCRATCH_BYTES (more than 256 samples
 * with 8 n_chan N^2 bytes above it), under MOFF_AUTOCORR_UV, or on a device
 * ordinal of 64 or more.
 */
#define MOFF_NOALLOC_SCRATCH_BYTES (128u << 20)
moff_status moff_image_noalloc(moff_plan plan, const void* E_dev, int64_t n_time,
                               const float* gains_dev, float* image_dev, void* hip_stream);

/*
 * Streaming form of the squaring and time averaging (Sec. 3, squaring at every
 * time stamp and accumulation over the integration): add the frames of E to
 * running sums.
 *   S_dev : float32 [n_chan][N][N], S += sum_t |Y|^2
 *   A_dev : float64 [n_chan][n_ktypes], A += sum_t sum_{a of type p} |e|^2
 *           (the self power that moff_finalize removes, Sec. 4.2)
 * E_dev, n_time, gains_dev as for moff_image.  accumulate(E1) then
 * accumulate(E2) equals accumulate(E1 ++ E2) up to rounding.  Within one call
 * |Y|^2 is summed in float32 over blocks of at most 256 samples per pixel and
 * the blocks in float64: one call adds at most 255 units of float32 rounding
 * (2^-24) relative to the summed power in the worst case, about 5 units
 * typically, however long the call; each call then rounds S once more, so a
 * caller streaming a long integration in many short calls adds one unit per
 * call (keep S in float64 on the caller's side, or make fewer, longer calls,
 * when that matters).
 * Errors: MOFF_ERR_INVALID_ARG for null or misaligned pointers or n_time < 1;
 * MOFF_ERR_UNSUPPORTED for a host-only plan or n_time * n_chan >= 2^31.
 */
moff_status moff_accumulate(moff_plan plan, const void* E_dev, int64_t n_time,
                            const float* gains_dev, float* S_dev, double* A_dev,
                            void* hip_stream);

/*
 * Self-power removal and averaging of streamed sums (Sec. 4.2: each antenna's
 * own power response, A[:, p] times P_p, is subtracted; Sec. 5,
 * eq. wt-dirty-image-EPIC for the pair normalisation):
 * image = (S - sum_p A[:, p] P_p) / n_time_total (times 1/(n_ant(n_ant-1)) with
 * MOFF_NORM_PAIRS; without the subtraction under MOFF_AUTOCORR_NONE; the
 * uv-plane rule under MOFF_AUTOCORR_UV).
 * S_dev, A_dev as produced by moff_accumulate; image_dev float32 [n_chan][N][N],
 * 16-byte aligned, overwritten.  n_time_total is any count >= 1 (it only scales).
 * Errors: MOFF_ERR_INVALID_ARG for null or misaligned pointers or
 * n_time_total < 1; MOFF_ERR_UNSUPPORTED for a host-only plan.
 */
moff_status moff_finalize(moff_plan plan, const float* S_dev, const double* A_dev,
                          int64_t n_time_total, float* image_dev, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Staged path: each step of the method as its own kernel with its result in
 * HBM.  Used to check each step against the oracle and as the plain baseline.
 * ------------------------------------------------------------------------- */

/*
 * Calibration + gridding (Sec. 3, E(r) = M(r,a) E(a)):
 *   eg_dev : complex64 [n_time][n_chan][N/2][N/2], Eg of every frame, overwritten.
 */
moff_status moff_grid(moff_plan plan, const void* E_dev, int64_t n_time,
                      const float* gains_dev, float* eg_dev, void* hip_stream);

/*
 * Self power of the calibrated fields:
 *   A_dev : float64 [n_chan][n_ktypes], A += sum_t sum_{a of type p} |g E|^2.
 */
moff_status moff_self_power(moff_plan plan, const void* E_dev, int64_t n_time,
                            const float* gains_dev, double* A_dev, void* hip_stream);

/*
 * Zero padding + 2-D transform of gridded frames (Sec. 3, spatial transform):
 *   eg_dev : complex64 [n_frames][N/2][N/2]
 *   y_dev  : complex64 [n_frames][N][N], Y[r][q] = sum Eg[iy][ix]
 *            exp(+2 pi i (iy (r - N/2) + ix (q - N/2)) / N), overwritten.
 */
moff_status moff_fft2(moff_plan plan, const float* eg_dev, int64_t n_frames,
                      float* y_dev, void* hip_stream);

/*
 * Squaring + time accumulation (Sec. 3, time averaging):
 *   y_dev : complex64 [n_time][n_chan][N][N]
 *   S_dev : float32 [n_chan][N][N], S += sum_t |Y|^2
 */
moff_status moff_detect_accumulate(moff_plan plan, const float* y_dev, int64_t n_time,
                                   float* S_dev, void* hip_stream);

/*
 * The staged pipeline end to end (grid -> fft2 -> detect -> finalize), in
 * time chunks through the plan's workspace; same output as moff_image.
 */
moff_status moff_image_staged(moff_plan plan, const void* E_dev, int64_t n_time,
                              const float* gains_dev, float* image_dev, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Visibility route (FX), for cross-checks of the MOFF image on the device.
 * ------------------------------------------------------------------------- */

/*
 * The same integration imaged by the paper's other method (Sec. 2): the pair
 * cross-products of the calibrated fields, V_ab = sum_t e_a conj(e_b) with
 * e = g E (eq. cc-vis), are gridded with each pair's power response -- the
 * cross-correlation of the two placed illumination tables (eq. e-field-conv) --
 * on the (2L - 1)^2 grid of footprint lags, L = grid_n / 2, and transformed
 * once per channel (eq. dirty-image-FX), in the pixel order of moff_image.
 *   E_dev, gains_dev, image_dev : as for moff_image.
 * The zero-spacing (a == b) terms are kept under MOFF_AUTOCORR_NONE and left
 * out otherwise, which is the exact self-power removal: the result then equals
 * moff_image's default image to rounding.  MOFF_AUTOCORR_UV and the
 * MOFF_MFMA_* flags do not apply here.  Arithmetic: 4+4-bit cross-products
 * are summed exactly in int32; complex64 cross-products are summed in float32
 * over chunks of 32 samples on the matrix cores and in float64 across chunks;
 * each pair's lag response is summed in float32, and binning, pair
 * combination and the transform's sums are float64.
 * MOFF_NORM_PAIRS scales as for moff_image.
 * Cost: O(n_chan (n_time n_ant^2 + n_ant^2 + N^2 log N)) work.  Channels run in
 * chunks whose workspace, 8 (n_ant^2 + (n_types^2 + 1) (2L - 1)^2 + (2L - 1) N)
 * bytes per channel, stays within about 2 GiB (at least one channel); it is
 * owned by the plan and shared with the plan's other entry points.  The pair
 * tables (about 2 n_ant^2 bytes: each unordered pair once) are built and
 * uploaded on the first call.
 * Errors: MOFF_ERR_INVALID_ARG for null or misaligned pointers or n_time < 1;
 * MOFF_ERR_UNSUPPORTED for a plan without a device, or 4+4-bit samples with
 * n_time > 2^24 (their cross-products are exact int32 sums on the matrix
 * cores);
 * MOFF_ERR_NOMEM when the workspace cannot be allocated; MOFF_ERR_HIP for a
 * failed launch.
 */
moff_status moff_image_fx(moff_plan plan, const void* E_dev, int64_t n_time,
                          const float* gains_dev, float* image_dev, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Gain gradient (calibration feedback, Sec. 3 "Calibration"; the image is
 * differentiable in the complex gains applied before gridding).
 * ------------------------------------------------------------------------- */

/*
 * Vector-Jacobian product of moff_image with respect to the gains:
 *   dL_dimage_dev : float32 [n_chan][N][N], R = dL/dI for a real loss L
 *   dL_dgains_dev : complex64 [n_chan][n_ant], overwritten with
 *                   dL/dRe(g) + i dL/dIm(g) = 2 dL/d(conj g)   (torch's convention)
 * E_dev, n_time, gains_dev (NULL = unit gains) as for moff_image.  With
 * e = g E and Y_t the image field of sample t,
 *   grad_a = (2 s / T) sum_t conj(E_ta) [ sum_{taps} conj(K_a) Z_t - e_ta rho_p(a) ],
 *   Z_t = adjoint 2-D DFT of R * Y_t on the aperture cells,  rho_p = sum_pix R P_p,
 * s the pair normalisation (1 unless MOFF_NORM_PAIRS), the rho term absent under
 * MOFF_AUTOCORR_NONE.  Under MOFF_AUTOCORR_UV the rho term is absent and R is
 * first shifted per channel by sum_pix R Pn / (N^2 a[0]) (the derivative of the
 * zero-spacing rule).  Every frame's grid and field are recomputed, never
 * stored for the whole integration; the sums over time are float64.
 * moff_gain_vjp runs one fused kernel in which each frame's grid, field and
 * adjoint stay on chip (when the plan's antennas fit its per-lane slots:
 * n_ant <= 4 x the workgroup size; otherwise it falls back to the staged form).
 * moff_gain_vjp_staged computes the same gradient with the steps separated by
 * HBM buffers, in time chunks through the plan workspace.  With timing enabled,
 * the HIP events bracket the fused adjoint kernel.
 */
moff_status moff_gain_vjp(moff_plan plan, const void* E_dev, int64_t n_time, const float* gains_dev,
                          const float* dL_dimage_dev, float* dL_dgains_dev, void* hip_stream);
moff_status moff_gain_vjp_staged(moff_plan plan, const void* E_dev, int64_t n_time, const float* gains_dev,
                                 const float* dL_dimage_dev, float* dL_dgains_dev, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MOFF_H */
