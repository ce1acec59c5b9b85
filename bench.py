"""Throughput of the fused MOFF imaging path on one MI355X.

A step images one integration of the HERA-shaped workload: 350 dishes on a
hexagonal grid of 14.6 m pitch, 7x7 Airy-like illumination tables, 1024
channels over 100-200 MHz, 256 time samples of 4+4-bit complex input, 256 x 256
padded grid: 262,144 frames per step (gridding, padded 2-D FFT, squaring,
accumulation and self-power removal for every (time, channel) frame), all
channels in one autotuned launch.  Inputs are synthetic, seeded, and resident
in HBM before timing starts.  The line also carries, in `extra`, the time of
the fused gain adjoint (moff_gain_vjp) on the calibration workload (1024
antennas, 256 channels, 128 samples, 256 grid, complex64 with gains).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--staged]
                    [--config 1..5] [--precision f32|f16|bf16] [--adjoint] [--fx]
                    [--adjoint-config 0..5] [--launch V,S]

--config picks another workload (2: LWA-shaped, 128 grid; 5: calibration).
--precision f16 / bf16 runs the reduced-precision path (16-bit gridded fields,
dense DFT on the matrix cores, float32 accumulation; grid 64 or 128) and also
times the float32 path on the same input; the CPU-baseline leg's oracle images
then give the per-image error of both.  The CPU leg also times the oracle on
one core and the paper's own CPU form of the pipeline (sparse gridding matrix
+ scipy.fft, float64 and float32, all cores and one), in `extra`.  --fx also
times the visibility route (moff_image_fx: correlate all antenna pairs, grid
the visibilities, one transform per channel) on the same input, the method
MOFF is compared with in the paper.  --adjoint times the gain adjoint on the
benchmark workload itself; --adjoint-config 0 skips the calibration-workload
adjoint.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (spec sheet)
PEAK_MFMA_16BIT_TFLOPS = 2500.0   # MI355X dense fp16 / bf16 matrix peak (spec sheet)

# HBM traffic per launch of the timed kernel, measured with rocprofv3 --pmc
# FETCH_SIZE and, in a second run, WRITE_SIZE on this script with the autotuner
# on, so that every candidate launch shape is counted (KiB per dispatch; the
# commands are in profiles/fused_kernel_hera_n256.md).  Scaled by what the same
# counters read for one 256 MiB device copy in the same runs (FETCH_SIZE
# 131,088-131,094 KiB, WRITE_SIZE 262,144 KiB).  All entries are from one set of runs on
# the current sources.  Keyed by (workload, precision, shape variant,
# workgroups); valid only for the kernel sources they were measured on,
# identified by TRAFFIC_SOURCES_SHA (KERNEL_SOURCES).
TRAFFIC_SOURCES_SHA = "e4f70da47563606b"
FETCH_SCALE, WRITE_SCALE = 262144.0 / 131093.0, 1.0
TRAFFIC_KIB = {
    (2, "f32", 0, 256): (25802, 57728),
    (2, "f32", 0, 512): (33537, 49922),
    (2, "f32", 0, 1024): (17279, 34308),
    (2, "f32", 0, 2048): (17534, 68562),
    (2, "f32", 0, 3072): (17787, 102787),
    (2, "f32", 0, 4096): (17891, 137051),
    (2, "f32", 0, 8192): (17492, 273957),
    (2, "f32", 0, 16384): (17334, 548572),
    (2, "f32", 1, 128): (25488, 57344),
    (2, "f32", 1, 256): (33167, 49154),
    (2, "f32", 1, 512): (16802, 32772),
    (2, "f32", 1, 1024): (16905, 65544),
    (2, "f32", 1, 1536): (16820, 98316),
    (2, "f32", 1, 2048): (16871, 131088),
    (2, "f32", 1, 4096): (16931, 262176),
    (2, "f32", 1, 8192): (17274, 524352),
    (3, "f32", 0, 4096): (54035, 262144),
    (3, "f32", 0, 8192): (50060, 524304),
    (3, "f32", 0, 16384): (50853, 1048609),
    (3, "f32", 0, 32768): (52323, 2097217),
    (3, "f32", 0, 65536): (58021, 4194433),
    (3, "f32", 0, 131072): (73561, 8388866),
    (3, "f32", 0, 262144): (1486197, 16777747),
    (3, "f32", 1, 2048): (70928, 286676),
    (3, "f32", 1, 4096): (60810, 573356),
    (3, "f32", 1, 8192): (102210, 1146896),
    (3, "f32", 1, 16384): (163573, 2293809),
    (3, "f32", 1, 32768): (319042, 4587654),
    (3, "f32", 1, 65536): (656732, 9175348),
    (3, "f32", 1, 131072): (1296538, 18350714),
    (4, "bf16", 0, 128): (129004, 8192),
    (4, "bf16", 0, 256): (128441, 16393),
    (4, "bf16", 0, 512): (128653, 32785),
    (4, "bf16", 0, 768): (128866, 49177),
    (4, "bf16", 0, 1024): (129079, 65569),
    (4, "bf16", 0, 2048): (129616, 131136),
    (4, "bf16", 0, 4096): (129734, 262272),
    (4, "bf16", 0, 8192): (130841, 524546),
    (4, "f16", 0, 128): (129019, 8192),
    (4, "f16", 0, 256): (128460, 16392),
    (4, "f16", 0, 512): (128672, 32784),
    (4, "f16", 0, 768): (128885, 49177),
    (4, "f16", 0, 1024): (129098, 65569),
    (4, "f16", 0, 2048): (129633, 131137),
    (4, "f16", 0, 4096): (129757, 262272),
    (4, "f16", 0, 8192): (130846, 524544),
    (4, "f32", 0, 256): (137860, 57728),
    (4, "f32", 0, 512): (145601, 49922),
    (4, "f32", 0, 1024): (129344, 34308),
    (4, "f32", 0, 2048): (129634, 68616),
    (4, "f32", 0, 3072): (129903, 102924),
    (4, "f32", 0, 4096): (130175, 137232),
    (4, "f32", 0, 8192): (131174, 274464),
    (4, "f32", 0, 16384): (133180, 548853),
    (4, "f32", 1, 128): (137537, 57344),
    (4, "f32", 1, 256): (145210, 49154),
    (4, "f32", 1, 512): (128915, 32772),
    (4, "f32", 1, 1024): (129386, 65544),
    (4, "f32", 1, 1536): (129854, 98316),
    (4, "f32", 1, 2048): (130301, 131088),
    (4, "f32", 1, 4096): (131640, 262176),
    (4, "f32", 1, 8192): (130414, 524352),
    (5, "f32", 0, 1024): (158456, 65536),
    (5, "f32", 0, 2048): (150892, 131080),
    (5, "f32", 0, 4096): (160215, 262160),
    (5, "f32", 0, 8192): (143492, 524320),
    (5, "f32", 0, 16384): (151870, 1048640),
    (5, "f32", 0, 32768): (168397, 2097280),
    (5, "f32", 0, 65536): (201060, 4194560),
    (5, "f32", 1, 512): (150456, 79360),
    (5, "f32", 1, 1024): (152983, 158729),
    (5, "f32", 1, 2048): (174530, 317458),
    (5, "f32", 1, 4096): (217594, 634913),
    (5, "f32", 1, 8192): (303225, 1269824),
    (5, "f32", 1, 16384): (474974, 2539648),
    (5, "f32", 1, 32768): (818068, 5079296),
}


# Sources that define the timed kernels and their tables (not the launch logic).
KERNEL_SOURCES = ("dft.h", "frame.h", "ingest.h", "kernels.h", "kernels.hip", "mfma.hip", "plan.cpp", "plan.h",
                  "shape.h")


def library_sources_sha():
    import hashlib
    m = hashlib.sha256()
    for name in KERNEL_SOURCES:
        m.update(name.encode())
        with open(os.path.join(ROOT, "paper_1510_08318_amd", "csrc", name), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(config, prec, launch, default_grid):
    """HBM bytes per launch from the recorded counters, or None when this
    launch or these sources were not profiled."""
    if not default_grid or library_sources_sha() != TRAFFIC_SOURCES_SHA:
        return None
    kib = TRAFFIC_KIB.get((config, prec, launch["variant"], launch["grid"]))
    if kib is None:
        return None
    return int(round((kib[0] * FETCH_SCALE + kib[1] * WRITE_SCALE) * 1024))


def adjoint_frame_flops(N, nnz):
    """Algorithmic work per frame of the gain adjoint: the forward transform and
    its adjoint (2 x 5 N^2 log2 N^2, Sec. 6.1 convention), gridding and
    degridding (8 flops per tap each) and the pixel-wise product R * Y
    (2 flops per pixel)."""
    return 2 * 5 * N * N * math.log2(N * N) + 16 * nnz + 2 * N * N


def time_adjoint_workload(cfg, steps):
    """Tuned fused gain adjoint (moff_gain_vjp) on workload `cfg`: ms per call
    between events on the current stream, the fused kernel's own duration (plan
    events) and its algorithmic rate."""
    import numpy as np
    import torch
    import paper_1510_08318_amd as moff
    import synth
    w = synth.make_config(cfg)
    T, C, Na = w.E.shape
    N = w.geom.grid_n
    dev = "cuda:0"
    E = torch.from_numpy(w.E).to(dev)
    g = torch.from_numpy(w.gains).to(dev) if w.gains is not None else \
        torch.ones((C, Na), dtype=torch.complex64, device=dev)
    plan = moff.Plan.from_geometry(w.geom, device=0)
    plan.autotune(E, g)                       # image launch and the adjoint's register budget
    R = torch.randn((C, N, N), dtype=torch.float32, device=dev, generator=torch.Generator(dev).manual_seed(7))
    grad = torch.empty((C, Na), dtype=torch.complex64, device=dev)
    plan.gain_vjp(E, g, R, out=grad)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    reps = max(3, min(steps, 10))
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    a0.record(stream)
    for _ in range(reps):
        plan.gain_vjp(E, g, R, out=grad)
    a1.record(stream)
    torch.cuda.synchronize()
    ms = a0.elapsed_time(a1) / reps
    plan.set_timing(True)
    kms = []
    for _ in range(reps):
        plan.gain_vjp(E, g, R, out=grad)
        kms.append(plan.last_kernel_ms())
    plan.set_timing(False)
    torch.cuda.synchronize()
    k_ms = float(np.mean(kms))
    nnz = int(sum(w.geom.ktype_k[t] ** 2 for t in w.geom.ant_ktype))
    flops = adjoint_frame_flops(N, nnz) * T * C
    out = {"workload": workload_name(cfg), "ms": round(ms, 4), "kernel_ms": round(k_ms, 4),
           "frames_per_s": T * C / (ms / 1e3), "waves_per_simd": plan.adjoint_waves()[0],
           "algorithmic_flops_per_frame": adjoint_frame_flops(N, nnz),
           "achieved_tflops": flops / (k_ms / 1e3) / 1e12,
           "frac_of_fp32_peak": flops / (k_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS}
    plan.close()
    del E, g, R, grad
    torch.cuda.empty_cache()
    return out


def workload_name(cfg):
    import synth
    return synth.CONFIG_NAMES[cfg]


def frame_flops(N, nnz):
    """Algorithmic work per frame: the FFT count 5 N^2 log2 N^2 for the padded
    grid (Sec. 6.1 cost convention, beta = 5), a complex multiply-add per gridding
    tap (8 flops) and |Y|^2 plus accumulation (4 flops per pixel)."""
    return 5 * N * N * math.log2(N * N) + 8 * nnz + 4 * N * N


def mfma_frame_flops(N):
    """Matrix-core work per frame of the reduced-precision path, L = N / 2.  Each
    stage runs over the base half of its phase vectors (the other half are
    their conjugates) as four real products: the row stage 4 x (L x L by L x L),
    the column stage 4 x (L x L by L x N), 8 L^2 (L + N) flops."""
    L = N // 2
    return 8 * L * L * (L + N)


def dense_dft_frame_flops(N):
    """The same transform as plain complex matrix products over the padded grid's
    nonzero half (no conjugate pairing): 8 L N (L + N) flops, L = N / 2."""
    L = N // 2
    return 8 * L * N * (L + N)


def cpu_baseline(w, budget_s=10.0):
    """The FP64 oracle timed on the host on a bounded sample of the same workload:
    whole channels (all time samples) in channel order until about budget_s of CPU
    work has been done; frames/s = frames imaged / seconds.  Also returns the
    oracle images and mean squared fields of the sampled channels."""
    import numpy as np
    import oracle
    threads = None
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max(int(i.get("num_threads", 1)) for i in info) if info else None
    except Exception:
        threads = None
    P = oracle.plan(w.geom)
    T = w.E.shape[0]
    oracle.moff_channel(w.geom, w.E[:2], w.gains, 0, P)      # warm BLAS threads
    t0 = time.perf_counter()
    n = 0
    images = []
    while n < w.E.shape[1]:
        img, parts = oracle.moff_channel(w.geom, w.E, w.gains, n, P, keep=True)
        images.append((n, img, parts["S"] / T))
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    del parts
    line = {"value": n * T / dt, "unit": "frames/s", "cores": threads or os.cpu_count(), "kind": "oracle",
            "sample": f"{n} channel(s) x all {T} time samples of the same workload "
                      f"({n * T} frames, {dt:.1f} s, float64 NumPy oracle)"}
    return line, images


def oracle_single_core(w, budget_s=3.0):
    """The FP64 oracle on one host core (BLAS limited to one thread): whole
    channels until about budget_s; frames/s."""
    import oracle
    from threadpoolctl import threadpool_limits
    P = oracle.plan(w.geom)
    T = w.E.shape[0]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        n = 0
        while n < w.E.shape[1]:
            oracle.moff_channel(w.geom, w.E, w.gains, n, P)
            n += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        dt = time.perf_counter() - t0
    return {"value": n * T / dt, "unit": "frames/s", "cores": 1, "sample": f"{n} channel(s) x {T} samples, {dt:.1f} s"}


def cpu_pipeline(w, plan, ref_images, budget_s=2.5):
    """The paper's own CPU form of the pipeline (Sec. 3: gridding as one sparse
    matrix product per readout, then the 2-D FFT of the zero-padded grid,
    squaring, accumulation and self-power removal), written with SciPy: a CSR
    gridding matrix from the plan's cells and tables, scipy.fft with the
    positive exponent and no normalisation, pixel N/2 at the phase centre.
    Timed in float64 and float32, on all host cores and on one, over whole
    channels (all time samples) until about budget_s per variant; the first
    sampled channel is checked against the oracle image of the CPU-baseline
    leg.  Context for the CPU baseline, not the target."""
    import numpy as np
    import scipy.fft as sfft
    import scipy.sparse as sp
    import synth
    from threadpoolctl import threadpool_limits
    g = w.geom
    Na, N, T, C = g.n_ant, g.grid_n, w.E.shape[0], g.n_chan
    L = N // 2
    nt = len(g.ktype_k)
    cells = plan.cells()
    rows, cols, vals = [], [], []
    for a in range(Na):
        K = np.asarray(g.ktype_vals[int(g.ant_ktype[a])], np.complex128)
        k = K.shape[0]
        ix0, iy0 = int(cells[a, 0]), int(cells[a, 1])
        for u in range(k):
            for v in range(k):
                rows.append((iy0 + u) * L + ix0 + v)
                cols.append(a)
                vals.append(K[u, v])
    W = sp.csr_matrix((np.asarray(vals), (rows, cols)), shape=(L * L, Na))
    Pp = np.stack([plan.power_pattern(p) for p in range(nt)])
    types = np.asarray(g.ant_ktype)
    ci4 = bool(g.flags & synth.IN_CI4)
    pairs = bool(g.flags & synth.NORM_PAIRS)

    def field(c, dt):
        x = w.E[:, c, :]
        if ci4:
            b = x.view(np.int8)
            e = (b >> 4).astype(np.float64) + 1j * ((b << 4).astype(np.int8) >> 4).astype(np.float64)
        else:
            e = x.astype(np.complex128)
        if w.gains is not None:
            e = e * w.gains[c][None, :]
        return e.astype(dt)

    def channel(c, dt, workers):
        e = field(c, dt)
        grid = np.zeros((T, N, N), dt)
        grid[:, :L, :L] = (W.astype(dt) @ e.T).T.reshape(T, L, L)
        Y = sfft.fftshift(sfft.ifft2(grid, axes=(1, 2), norm="forward", workers=workers), axes=(1, 2))
        S = (Y.real.astype(np.float64) ** 2 + Y.imag.astype(np.float64) ** 2).sum(0)
        A = np.array([(np.abs(e[:, types == p].astype(np.complex128)) ** 2).sum() for p in range(nt)])
        img = (S - np.tensordot(A, Pp, 1)) / T
        return img / (Na * (Na - 1)) if pairs else img

    ncores = os.cpu_count() or 1
    out = {}
    for name, dt in (("f64", np.complex128), ("f32", np.complex64)):
        for cores in (ncores, 1):
            with threadpool_limits(limits=cores):
                channel(0, dt, cores)   # warm-up
                t0 = time.perf_counter()
                n = 0
                while n < C:
                    channel(n, dt, cores)
                    n += 1
                    if time.perf_counter() - t0 >= budget_s:
                        break
                dt_s = time.perf_counter() - t0
            out[f"scipy_{name}_{cores}core"] = {"value": n * T / dt_s, "unit": "frames/s", "cores": cores,
                                                "sample": f"{n} channel(s) x {T} samples, {dt_s:.1f} s"}
    if ref_images:
        c, ref, pbar = ref_images[0]
        for name, dt in (("f64", np.complex128), ("f32", np.complex64)):
            d = channel(c, dt, ncores) - ref
            out[f"scipy_{name}_err_inf_vs_oracle"] = float(f"{np.abs(d).max() / np.abs(pbar).max():.3g}")
    return out


def image_errors(img, ref_images):
    """Per sampled channel (one image each): err_inf = max|dI| / max|Pbar| and
    err_2 = ||dI|| / ||Pbar||, reported per image (3 significant digits) and as
    maxima over the sample."""
    import numpy as np
    chans, e_inf, e_2 = [], [], []
    for c, ref, pbar in ref_images:
        d = img[c].astype(np.float64) - ref
        chans.append(int(c))
        e_inf.append(float(np.abs(d).max() / np.abs(pbar).max()))
        e_2.append(float(np.linalg.norm(d) / np.linalg.norm(pbar)))
    sig = lambda v: float(f"{v:.3g}")
    return {"images": len(chans), "channels": f"{chans[0]}-{chans[-1]}" if chans else "",
            "err_inf_max": sig(max(e_inf)) if e_inf else None, "err_2_max": sig(max(e_2)) if e_2 else None,
            "err_inf": [sig(v) for v in e_inf], "err_2": [sig(v) for v in e_2]}


def time_plan(plan, E, gains, out, steps, warmup, tune):
    """(ms per step, mean fused-kernel ms, launch configuration).  The timed
    steps run back to back on the current stream between two events; kernel
    durations come from a second pass with per-call kernel events."""
    import numpy as np
    import torch
    T = E.shape[0]
    if tune:
        plan.autotune(E, gains)
    launch = plan.config(T)
    for _ in range(warmup):
        plan.image(E, gains, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.image(E, gains, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / steps
    plan.set_timing(True)
    kernel_ms = []
    for _ in range(steps):
        plan.image(E, gains, out=out)
        kernel_ms.append(plan.last_kernel_ms())
    plan.set_timing(False)
    torch.cuda.synchronize()
    return ms_per_step, float(np.mean(kernel_ms)), launch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--staged", action="store_true", help="also time the staged (per-step HBM) pipeline")
    ap.add_argument("--fx", action="store_true", help="also time the visibility (FX) route on the same input")
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--grid", type=int, default=0, help="override the workload's grid size")
    ap.add_argument("--precision", choices=("f32", "f16", "bf16"), default=None,
                    help="f32: float32 FFT path; f16 / bf16: matrix-core DFT path (default: f16 for config 4)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch autotuner (heuristic configuration)")
    ap.add_argument("--launch", default="", help="fixed launch shape 'variant,slices' instead of the autotuner")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the gain adjoint (moff_gain_vjp) on the same workload")
    ap.add_argument("--adjoint-config", type=int, default=5,
                    help="workload on which the fused gain adjoint is timed for `extra` (0: skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; channels shard across GPUs "
                                   "with no exchange, so a multi-GPU figure is not measured here"}))
        sys.exit(2)
    prec = args.precision or ("f16" if args.config == 4 else "f32")

    import torch
    import paper_1510_08318_amd as moff
    import synth

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = synth.make_config(args.config, grid_n=args.grid or None)
    T, C, Na = w.E.shape
    N = w.geom.grid_n
    dev = "cuda:0"
    E = torch.from_numpy(w.E).to(dev)
    gains = torch.from_numpy(w.gains).to(dev) if w.gains is not None else None
    extra_flags = {"f32": 0, "f16": synth.MFMA_F16, "bf16": synth.MFMA_BF16}[prec]
    plan = moff.Plan.from_geometry(w.geom, device=0, extra_flags=extra_flags)
    out = torch.empty((C, N, N), dtype=torch.float32, device=dev)
    nnz = int(sum(w.geom.ktype_k[t] ** 2 for t in w.geom.ant_ktype))
    frames = T * C
    stream = torch.cuda.current_stream()

    if args.launch:
        v, sl = (int(x) for x in args.launch.split(","))
        plan.set_config(v, sl)
    tune = not (args.no_tune or args.launch)
    ms_per_step, k_ms, launch = time_plan(plan, E, gains, out, args.steps, args.warmup, tune)
    value = frames / (ms_per_step / 1e3)
    extra = {"fused_kernel_ms": round(k_ms, 4), "frames_per_step": frames,
             "algorithmic_flops_per_frame": frame_flops(N, nnz)}
    traffic = measured_traffic(args.config, prec, launch, args.grid == 0)
    if traffic is not None:
        extra["traffic_GBps"] = traffic / (k_ms / 1e3) / 1e9
    if prec == "f32":
        achieved = frame_flops(N, nnz) * frames / (k_ms / 1e3) / 1e12
        roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic}
    else:
        extra["mfma_flops_per_frame"] = mfma_frame_flops(N)
        achieved = mfma_frame_flops(N) * frames / (k_ms / 1e3) / 1e12
        extra["dense_dft_equivalent_tflops"] = round(dense_dft_frame_flops(N) * frames / (k_ms / 1e3) / 1e12, 1)
        roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_16BIT_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_MFMA_16BIT_TFLOPS, "traffic": traffic}
        plan32 = moff.Plan.from_geometry(w.geom, device=0)
        out32 = torch.empty_like(out)
        ms32, k32, launch32 = time_plan(plan32, E, gains, out32, args.steps, args.warmup, not args.no_tune)
        plan32.close()
        extra["f32_fft_ms_per_step"] = round(ms32, 4)
        extra["f32_fft_kernel_ms"] = round(k32, 4)
        extra["f32_fft_frames_per_s"] = frames / (ms32 / 1e3)
        extra["speedup_vs_f32_fft"] = round(ms32 / ms_per_step, 3)

    if args.staged:
        out2 = torch.empty_like(out)
        plan.image_staged(E, gains, out=out2)
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(3):
            plan.image_staged(E, gains, out=out2)
        s1.record(stream)
        torch.cuda.synchronize()
        st_ms = s0.elapsed_time(s1) / 3
        extra["staged_ms_per_step"] = round(st_ms, 3)
        extra["fused_speedup_vs_staged"] = round(st_ms / ms_per_step, 2)
        extra["staged_vs_fused_max_abs_diff"] = float((out2 - out).abs().max().item())

    if args.fx:
        out3 = torch.empty_like(out)
        plan.image_fx(E, gains, out=out3)
        torch.cuda.synchronize()
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(3):
            plan.image_fx(E, gains, out=out3)
        f1.record(stream)
        torch.cuda.synchronize()
        fx_ms = f0.elapsed_time(f1) / 3
        extra["fx_ms_per_step"] = round(fx_ms, 3)
        extra["fx_frames_per_s"] = frames / (fx_ms / 1e3)
        extra["moff_speedup_vs_fx"] = round(fx_ms / ms_per_step, 2)
        extra["fx_vs_moff_max_abs_diff_rel"] = float((out3 - out).abs().max().item() / out.abs().max().item())

    if args.adjoint:
        g_in = gains if gains is not None else torch.ones((C, Na), dtype=torch.complex64, device=dev)
        R = torch.randn((C, N, N), dtype=torch.float32, device=dev)
        reps = max(2, min(args.steps, 5))
        grads = {}
        for staged in (False, True):
            grad = torch.empty((C, Na), dtype=torch.complex64, device=dev)
            plan.gain_vjp(E, g_in, R, out=grad, staged=staged)
            torch.cuda.synchronize()
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            for _ in range(reps):
                plan.gain_vjp(E, g_in, R, out=grad, staged=staged)
            a1.record(stream)
            torch.cuda.synchronize()
            ms = a0.elapsed_time(a1) / reps
            key = "adjoint_staged" if staged else "adjoint"
            extra[key + "_ms_per_step"] = round(ms, 3)
            extra[key + "_frames_per_s"] = frames / (ms / 1e3)
            grads[staged] = grad
        plan.set_timing(True)
        plan.gain_vjp(E, g_in, R, out=grads[False])
        extra["adjoint_kernel_ms"] = round(plan.last_kernel_ms(), 4)
        extra["adjoint_waves_per_simd"] = plan.adjoint_waves()[0]
        plan.set_timing(False)
        extra["adjoint_fused_vs_staged_max_rel_diff"] = float(
            ((grads[False] - grads[True]).abs().max() / grads[True].abs().max()).item())

    if args.adjoint_config:
        extra["adjoint_ms"] = None
        adj = time_adjoint_workload(args.adjoint_config, args.steps)
        extra["adjoint_ms"] = adj["ms"]
        extra["adjoint_calibration"] = adj

    cpu = None
    if not args.no_cpu:
        cpu, ref_images = cpu_baseline(w)
        img = out.cpu().numpy()
        extra["error_vs_oracle"] = {prec: image_errors(img, ref_images)}
        if prec != "f32":
            extra["error_vs_oracle"]["f32"] = image_errors(out32.cpu().numpy(), ref_images)
        extra["cpu_oracle_1core"] = oracle_single_core(w)
        extra["cpu_pipeline"] = cpu_pipeline(w, plan, ref_images)
        del ref_images

    line = {
        "metric": "MOFF frames/s (grid\u00d7channels per time sample) + % HBM roofline; adjoint ms",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic (seeded point-source sky + Gaussian noise" + (", 4+4-bit quantised)" if (w.geom.flags & synth.IN_CI4) else ")"),
        "config": {"workload": synth.CONFIG_NAMES[args.config],
                   "n_ant": Na, "n_chan": C, "n_time": T, "grid": N,
                   "input": "ci4" if (w.geom.flags & synth.IN_CI4) else "c64",
                   "launch": {k: launch[k] for k in ("variant", "slices", "grid", "threads", "tuned")}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
