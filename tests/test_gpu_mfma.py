"""GPU: the reduced-precision path (MOFF_MFMA_F16 / MOFF_MFMA_BF16, 16-bit gridded
fields and matrix-core DFT with float32 accumulation) against the FP64 oracle.

Stated bound, with u the unit roundoff of the 16-bit format (2^-11 binary16,
2^-8 bfloat16) and the error metrics of the float32 parity tests (per channel,
relative to the oracle's mean squared field Pbar = S / T):
    err_inf = max |I - I_oracle| / max |Pbar|  <= 16 u
    err_2   = ||I - I_oracle||_2 / ||Pbar||_2  <= 4 u
Derivation: each of the four roundings on the path (gridded field, row-stage
phase factors, row-stage output, column-stage phase factors) perturbs Y by a
relative amount of at most u per component, so |dY| <~ 2 u |Y|_rms per frame and
|d|Y|^2| <~ 4 u |Y| |Y|_rms; errors that are independent from frame to frame
average down, the phase-factor errors do not.  Relative to Pbar (whose
average over pixels is |Y|_rms^2 by Parseval) that gives err_2 ~ 4 u in the worst
(fully systematic) case; err_inf allows a further factor of 4 for the largest
pixel of a 128 x 128 image.  Each test also checks the float32 path on the same
input to 1e-5, so the reported error is the precision's, not the input's.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
PREC = {"f16": (synth.MFMA_F16, 2.0 ** -11), "bf16": (synth.MFMA_BF16, 2.0 ** -8)}


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def moff():
    import paper_1510_08318_amd as m
    m._lib.lib()   # raises if the library is missing: no fallback
    return m


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def oracle_channels(w, channels):
    """Oracle images and the reference scale of the error metric, Pbar = S / T,
    carrying the image's own pair normalisation 1 / (N_a (N_a - 1)) when that
    flag is set (Sec. 4), so the metric is relative to the image's scale."""
    P = oracle.plan(w.geom)
    na = w.geom.n_ant
    norm = 1.0 / (na * (na - 1)) if int(w.geom.flags) & synth.NORM_PAIRS else 1.0
    imgs, pbar = [], []
    for c in channels:
        img, parts = oracle.moff_channel(w.geom, w.E, w.gains, c, P, keep=True)
        imgs.append(img)
        pbar.append(parts["S"] / w.E.shape[0] * norm)
    return np.stack(imgs), np.stack(pbar)


def errors(got, ref, pbar):
    out = []
    for c in range(ref.shape[0]):
        d = got[c].astype(np.float64) - ref[c]
        out.append((float(np.abs(d).max() / np.abs(pbar[c]).max()), float(np.linalg.norm(d) / np.linalg.norm(pbar[c]))))
    return out


def run_image(torch, moff, w, extra_flags=0, slices=None):
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=extra_flags) as p:
        if slices is not None:
            p.set_config(0, slices)
        out = p.image(to_dev(torch, w.E), to_dev(torch, w.gains) if w.gains is not None else None)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def report(label, prec, errs):
    """Per-image error lines; also appended to $MOFF_ERROR_REPORT (JSON lines) if set."""
    path = os.environ.get("MOFF_ERROR_REPORT")
    for c, (ei, e2) in enumerate(errs):
        print(f"[mfma-error] {label} {prec} image {c}: err_inf={ei:.3e} err_2={e2:.3e}")
        if path:
            with open(path, "a") as f:
                f.write(json.dumps({"case": label, "precision": prec, "image": c, "err_inf": ei, "err_2": e2}) + "\n")


def check(torch, moff, w, label, precs=("f16", "bf16"), channels=None, slices=None):
    C = w.geom.n_chan
    channels = list(range(C)) if channels is None else list(channels)
    ref, pbar = oracle_channels(w, channels)
    fp32 = run_image(torch, moff, w)[channels]
    e32 = errors(fp32, ref, pbar)
    report(label, "f32", e32)
    assert max(max(e) for e in e32) <= 1e-5
    for prec in precs:
        flag, u = PREC[prec]
        got = run_image(torch, moff, w, flag, slices)
        assert np.isfinite(got).all()
        errs = errors(got[channels], ref, pbar)
        report(label, prec, errs)
        for c, (ei, e2) in enumerate(errs):
            assert ei <= 16 * u and e2 <= 4 * u, f"{label} {prec} image {c}: err_inf={ei:.3g} err_2={e2:.3g}"


def _hetero(N, flags=0, fmt=synth.IN_C64):
    rng = np.random.default_rng(31 + N)
    w = synth.random_case(40 + N, 60, N, 2, 5, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 5)],
                          fmt=fmt, extent_m=0.35 * N, cell_m=1.0)
    w.geom.flags |= flags
    return w


CASES = {
    "config4_n128": lambda: synth.make_config(4, n_time=6, n_chan=2),
    "config4_n64": lambda: synth.make_config(4, n_time=6, n_chan=2, grid_n=64),
    "config2_n128_ci4": lambda: synth.make_config(2, n_time=5, n_chan=2),
    "config5_n128_gains": lambda: synth.make_config(5, n_time=3, n_chan=2, grid_n=128),
    "hetero_n64_ci4": lambda: _hetero(64, fmt=synth.IN_CI4),
    "hetero_n128_pairs": lambda: _hetero(128, flags=synth.NORM_PAIRS),
    "hetero_n64_autos": lambda: _hetero(64, flags=synth.AUTOCORR_NONE),
}


@pytest.mark.parametrize("case", list(CASES))
def test_mfma_image_vs_oracle(torch, moff, case):
    check(torch, moff, CASES[case](), case)


def test_mfma_slicing_and_accumulate(torch, moff):
    """Time slices (per-slice partial sums + ordered reduction) and split
    accumulation agree with one pass to float32 rounding: the transform of a
    frame does not depend on how frames are grouped.  Slices of one and two
    frames run the kernel's frame pipeline shorter than its depth."""
    w = synth.make_config(4, n_time=9, n_chan=3, grid_n=64)
    flag = synth.MFMA_F16
    base = run_image(torch, moff, w, flag, slices=1)
    scale = np.abs(base).max()
    for sl in (2, 3, 4, 5, 9):
        got = run_image(torch, moff, w, flag, slices=sl)
        assert np.abs(got - base).max() <= 1e-5 * scale, sl
    import torch as t
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=flag) as p:
        E = to_dev(torch, w.E)
        C, N = w.geom.n_chan, w.geom.grid_n
        S = t.zeros((C, N, N), dtype=t.float32, device="cuda:0")
        A = t.zeros((C, w.geom.n_ktypes), dtype=t.float64, device="cuda:0")
        p.accumulate(E[:4], S, A)
        p.accumulate(E[4:], S, A)
        img = p.finalize(S, A, 9)
        torch.cuda.synchronize()
        assert np.abs(img.cpu().numpy() - base).max() <= 1e-5 * scale


def test_mfma_deterministic(torch, moff):
    w = synth.make_config(4, n_time=4, n_chan=2)
    a = run_image(torch, moff, w, synth.MFMA_BF16)
    b = run_image(torch, moff, w, synth.MFMA_BF16)
    assert np.array_equal(a, b)


def test_mfma_autotune(torch, moff):
    w = synth.make_config(4, n_time=20, n_chan=4, grid_n=64)
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=synth.MFMA_F16) as p:
        E = to_dev(torch, w.E)
        cfg = p.autotune(E)
        assert cfg["tuned"] and cfg["threads"] == 256 and cfg["n_variants"] == 1   # 2 matrix + 2 gather waves
        out = p.image(E)
        torch.cuda.synchronize()
        img = out.cpu().numpy()
    ref, pbar = oracle_channels(w, range(4))
    for ei, e2 in errors(img, ref, pbar):
        assert ei <= 16 * 2.0 ** -11 and e2 <= 4 * 2.0 ** -11


@pytest.mark.parametrize("N", [128, 64])
def test_mfma_full_size_sampled_channels(torch, moff, N):
    """The reduced-precision workload at full size (1000 samples x 128 channels),
    in the default launch configuration, checked on channels the oracle computes
    one by one."""
    w = synth.make_config(4, grid_n=N)
    check(torch, moff, w, f"config4_full_n{N}", channels=[0, 64, 127])
