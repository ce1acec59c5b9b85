"""Throughput of the fused MOFF imaging path on one MI355X.

A step images one integration of the LWA-shaped workload: 256 antennas in a
100 m disc, 3x3 dipole illumination, 128 channels over 40-80 MHz, 1000 time
samples of 4+4-bit complex input, 128 x 128 padded grid: 128,000 frames per step
(gridding, padded 2-D FFT, squaring, accumulation and self-power removal for every
(time, channel) frame).  Inputs are synthetic, seeded, and resident in HBM before
timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--staged]

Prints one JSON line.
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


def frame_flops(N, nnz):
    """Algorithmic work per frame: the FFT count 5 N^2 log2 N^2 for the padded
    grid (Sec. 6.1 cost convention, beta = 5), a complex multiply-add per gridding
    tap (8 flops) and |Y|^2 plus accumulation (4 flops per pixel)."""
    return 5 * N * N * math.log2(N * N) + 8 * nnz + 4 * N * N


def cpu_baseline(w, budget_s=10.0):
    """The FP64 oracle timed on the host on a bounded sample of the same workload:
    whole channels (all time samples) in channel order until about budget_s of CPU
    work has been done; frames/s = frames imaged / seconds."""
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
    while n < w.E.shape[1]:
        oracle.moff_channel(w.geom, w.E, w.gains, n, P)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n * T / dt, "unit": "frames/s", "cores": threads or os.cpu_count(), "kind": "oracle",
            "sample": f"{n} channel(s) x all {T} time samples of the same workload "
                      f"({n * T} frames, {dt:.1f} s, float64 NumPy oracle)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--staged", action="store_true", help="also time the staged (per-step HBM) pipeline")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true", help="skip the launch autotuner (heuristic configuration)")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the gain adjoint (moff_gain_vjp) on the same workload")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; channels shard across GPUs "
                                   "with no exchange, so a multi-GPU figure is not measured here"}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1510_08318_amd as moff
    import synth

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = synth.make_config(args.config)
    T, C, Na = w.E.shape
    N = w.geom.grid_n
    dev = "cuda:0"
    E = torch.from_numpy(w.E).to(dev)
    gains = torch.from_numpy(w.gains).to(dev) if w.gains is not None else None
    plan = moff.Plan.from_geometry(w.geom, device=0)
    out = torch.empty((C, N, N), dtype=torch.float32, device=dev)
    nnz = int(sum(w.geom.ktype_k[t] ** 2 for t in w.geom.ant_ktype))
    frames = T * C

    if not args.no_tune:
        plan.autotune(E, gains)
    launch = plan.config(T)
    for _ in range(args.warmup):
        plan.image(E, gains, out=out)
    torch.cuda.synchronize()

    plan.set_timing(True)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kernel_ms = []
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.image(E, gains, out=out)
        kernel_ms.append(plan.last_kernel_ms())
    ev1.record(stream)
    torch.cuda.synchronize()
    plan.set_timing(False)
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    k_ms = float(np.mean(kernel_ms))
    value = frames / (ms_per_step / 1e3)
    flops_launch = frame_flops(N, nnz) * frames
    achieved = flops_launch / (k_ms / 1e3) / 1e12

    extra = {"fused_kernel_ms": round(k_ms, 4), "frames_per_step": frames,
             "algorithmic_flops_per_frame": frame_flops(N, nnz)}
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

    if args.adjoint:
        g_in = gains if gains is not None else torch.ones((C, Na), dtype=torch.complex64, device=dev)
        R = torch.randn((C, N, N), dtype=torch.float32, device=dev)
        grad = torch.empty((C, Na), dtype=torch.complex64, device=dev)
        plan.gain_vjp(E, g_in, R, out=grad)
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        reps = max(2, min(args.steps, 5))
        a0.record(stream)
        for _ in range(reps):
            plan.gain_vjp(E, g_in, R, out=grad)
        a1.record(stream)
        torch.cuda.synchronize()
        extra["adjoint_ms_per_step"] = round(a0.elapsed_time(a1) / reps, 3)
        extra["adjoint_frames_per_s"] = frames / (a0.elapsed_time(a1) / reps / 1e3)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w)

    line = {
        "metric": "MOFF frames/s (grid x channels per time sample)",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded point-source sky + Gaussian noise" + (", 4+4-bit quantised)" if (w.geom.flags & synth.IN_CI4) else ")"),
        "config": {"workload": synth.CONFIG_NAMES[args.config],
                   "n_ant": Na, "n_chan": C, "n_time": T, "grid": N,
                   "input": "ci4" if (w.geom.flags & synth.IN_CI4) else "c64",
                   "launch": {k: launch[k] for k in ("variant", "slices", "grid", "threads", "tuned")}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
