"""GPU gain gradient (adjoint of the MOFF path) against the FP64 oracle gradient
and against finite differences of the FP64 oracle's forward image.

Tolerance: the GPU path computes the transforms in float32 and the sums over
time in float64; errors are measured relative to the largest gradient entry of
the channel, bound 1e-4 (the finite-difference bound asked of the adjoint).
"""
import zlib

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def moff():
    import paper_1510_08318_amd as m
    m._lib.lib()
    return m


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_grad(torch, moff, w, R, staged=False):
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        g = p.gain_vjp(dev(torch, w.E), dev(torch, w.gains), dev(torch, R.astype(np.float32)), staged=staged)
        torch.cuda.synchronize()
        return g.cpu().numpy().astype(np.complex128)


def rel_err(got, ref):
    return max(np.abs(got[c] - ref[c]).max() / np.abs(ref[c]).max() for c in range(ref.shape[0]))


def small(seed, N, n_ant, kernels, C=2, T=3, flags=0, fmt=synth.IN_C64, extent=3.0, cell=1.0):
    w = synth.random_case(seed, n_ant, N, C, T, kernels, fmt=fmt, extent_m=extent, cell_m=cell)
    w.geom.flags |= flags
    return w


CASES = {
    "n8": lambda r: small(1, 8, 4, [synth.random_kernel(r, 2)], extent=1.5),
    "n16_hetero": lambda r: small(2, 16, 7, [synth.random_kernel(r, 2), synth.random_kernel(r, 3)]),
    "n32_ci4": lambda r: small(3, 32, 12, [synth.random_kernel(r, 3)], fmt=synth.IN_CI4, extent=10.0),
    "n64_pairs": lambda r: small(4, 64, 20, [synth.random_kernel(r, 3)], flags=synth.NORM_PAIRS, extent=30.0),
    "n128_autos": lambda r: small(5, 128, 30, [synth.random_kernel(r, 3), synth.random_kernel(r, 5)],
                                  flags=synth.AUTOCORR_NONE, extent=80.0, cell=1.5),
    "config5_sub": lambda r: synth.make_config(5, n_time=3, n_chan=2),
    # more antennas than the fused kernel's per-lane slots hold at N = 32: the
    # gradient falls back to the staged form
    "n32_many_antennas": lambda r: small(9, 32, 300, [synth.random_kernel(r, 1)], extent=14.0),
}


@pytest.mark.parametrize("staged", [False, True], ids=["fused", "staged"])
@pytest.mark.parametrize("case", list(CASES))
def test_gradient_vs_oracle(torch, moff, case, staged):
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    w = CASES[case](np.random.default_rng(7))
    if w.gains is None:
        w.gains = synth.random_gains(rng, w.geom.n_chan, w.geom.n_ant)
    C, N = w.geom.n_chan, w.geom.grid_n
    R = rng.standard_normal((C, N, N)).astype(np.float32)
    ref = oracle.gain_gradient(w.geom, w.E, w.gains, R.astype(np.float64))
    got = gpu_grad(torch, moff, w, R, staged)
    err = rel_err(got, ref)
    assert err <= TOL, f"{case}: {err:.3g}"


def test_full_size_calibration_gradient_sampled(torch, moff):
    """The calibration workload at full size (256 channels, 128 samples, 1024
    antennas of two types, N = 256) through the fused adjoint, checked on channels
    the oracle computes one by one."""
    w = synth.make_config(5)
    C, N = w.geom.n_chan, w.geom.grid_n
    rng = np.random.default_rng(23)
    R = rng.standard_normal((C, N, N)).astype(np.float32)
    got = gpu_grad(torch, moff, w, R)
    assert np.isfinite(got).all()
    chans = [0, 131, 255]
    ref = oracle.gain_gradient(w.geom, w.E, w.gains, R[chans].astype(np.float64), channels=chans)
    assert rel_err(got[chans], ref) <= TOL


def fd_check(torch, moff, w, model, rng, n_random, label):
    """Directional derivatives of L(g) = sum (I - M)^2: the GPU adjoint against
    central differences of the oracle's float64 forward image (an
    implementation independent of both gradient codes).  Each direction must
    agree to 1e-4 of its own derivative, with a floor of 0.1 of the typical
    derivative size ||grad|| ||d|| / sqrt(n) for directions the gradient is
    nearly orthogonal to (there the float32 transforms' absolute error, about
    1e-7 of the largest entry, sets the limit).  Directions: random complex ones, and the real and
    imaginary part of single gains (the two largest gradient entries and one
    random antenna of each channel)."""
    g0 = w.gains.astype(np.complex128)
    L0, R = oracle.image_loss(w.geom, w.E, g0, model)
    got = gpu_grad(torch, moff, w, R)
    n = got.size
    dirs = [rng.standard_normal(g0.shape) + 1j * rng.standard_normal(g0.shape) for _ in range(n_random)]
    for c in range(g0.shape[0]):
        picks = list(np.argsort(-np.abs(got[c]))[:2]) + [int(rng.integers(g0.shape[1]))]
        for a in picks:
            for unit in (1.0, 1j):
                d = np.zeros(g0.shape, complex)
                d[c, a] = unit
                dirs.append(d)
    h = 1e-6
    for d in dirs:
        fd = (oracle.image_loss(w.geom, w.E, g0 + h * d, model)[0]
              - oracle.image_loss(w.geom, w.E, g0 - h * d, model)[0]) / (2 * h)
        an = float(np.real(np.sum(np.conj(got) * d)))
        floor = 0.1 * np.linalg.norm(got) * np.linalg.norm(d) / np.sqrt(n)
        assert abs(fd - an) <= TOL * max(abs(fd), floor), (label, fd, an, floor)


def test_gradient_vs_finite_differences(torch, moff):
    rng = np.random.default_rng(11)
    w = small(8, 32, 10, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 2)], extent=8.0)
    model = rng.standard_normal((2, 32, 32)) * 3.0
    fd_check(torch, moff, w, model, rng, 6, "heterogeneous n32")


def test_gradient_vs_finite_differences_calibration_layout(torch, moff):
    """The calibration layout (1024 antennas in a 400 m disc, 3x3 and 7x7
    tables, grid 256, complex64 samples through gains) on two channels and four
    samples."""
    rng = np.random.default_rng(12)
    w = synth.make_config(5, n_time=4, n_chan=2)
    model = rng.standard_normal((2, 256, 256)) * 0.1
    fd_check(torch, moff, w, model, rng, 3, "calibration layout")


def test_gauge_and_optimum(torch, moff):
    """Zero gradient at the true calibration of the calibration workload, and a
    gradient orthogonal to a common phase rotation elsewhere."""
    w = synth.make_config(5, n_time=4, n_chan=2)
    g_true = w.extra["g_true"].astype(np.complex128)
    E_sky = w.E.astype(np.complex128) / g_true[None]
    model = oracle.moff_image(w.geom, E_sky, None)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = dev(torch, w.E)
        out = {}
        for name, g in (("opt", 1.0 / g_true),
                        ("off", (1.0 / g_true) * (1 + 0.05 * np.random.default_rng(2).standard_normal(g_true.shape)))):
            gt = dev(torch, g.astype(np.complex64))
            img = p.image(E, gt)
            R = 2.0 * (img - dev(torch, model.astype(np.float32)))
            grad = p.gain_vjp(E, gt, R.contiguous())
            torch.cuda.synchronize()
            out[name] = (grad.cpu().numpy().astype(np.complex128), g)
    g_opt, _ = out["opt"]
    g_off, goff = out["off"]
    assert np.abs(g_opt).max() <= 1e-3 * np.abs(g_off).max()
    for c in range(2):
        v = np.sum(np.conj(g_off[c]) * goff[c])
        assert abs(v.imag) <= TOL * np.sum(np.abs(g_off[c]) * np.abs(goff[c]))


def test_autograd_function(torch, moff):
    rng = np.random.default_rng(3)
    w = synth.make_config(5, n_time=3, n_chan=2)
    model = rng.standard_normal((2, 256, 256)).astype(np.float32) * 10.0
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = dev(torch, w.E)
        gains = dev(torch, w.gains).requires_grad_(True)
        img = moff.moff_image_autograd(p, E, gains)
        loss = ((img - dev(torch, model)) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        got = gains.grad.cpu().numpy().astype(np.complex128)
        I = img.detach().cpu().numpy().astype(np.float64)
    R = 2.0 * (I - model)
    ref = oracle.gain_gradient(w.geom, w.E, w.gains, R)
    assert rel_err(got, ref) <= TOL


@pytest.mark.parametrize("case", ["config5_sub", "config3_sub", "n128_autos"])
def test_adjoint_register_budgets_agree(torch, moff, case):
    """The fused adjoint is built with several register budgets (waves per SIMD:
    1-2 at N = 256, 1-3 at N = 128; the excess spilled to accumulation registers
    or scratch memory): every budget gives the oracle gradient and the same
    result, the autotuner keeps one of them, and budgets outside 1 .. max are
    rejected.  complex64 samples with two table types (calibration layout),
    4+4-bit samples with 7x7 tables (HERA-shaped), and a heterogeneous N = 128
    case with the zero-spacing terms kept."""
    w = CASES[case](np.random.default_rng(7)) if case in CASES else synth.make_config(3, n_time=3, n_chan=2)
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 1)
    if w.gains is None:
        w.gains = synth.random_gains(rng, w.geom.n_chan, w.geom.n_ant)
    C, N = w.geom.n_chan, w.geom.grid_n
    R = rng.standard_normal((C, N, N)).astype(np.float32)
    ref = oracle.gain_gradient(w.geom, w.E, w.gains, R.astype(np.float64))
    wmax = {128: 3, 256: 2}[N]
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        assert p.adjoint_waves() == (1, wmax)
        E, g, Rd = dev(torch, w.E), dev(torch, w.gains), dev(torch, R)
        got = {}
        for wps in range(1, wmax + 1):
            p.set_adjoint_waves(wps)
            got[wps] = p.gain_vjp(E, g, Rd).cpu().numpy().astype(np.complex128)
            assert rel_err(got[wps], ref) <= TOL, f"{case} waves {wps}"
        scale = max(np.abs(got[1][c]).max() for c in range(C))
        for wps in range(2, wmax + 1):
            assert np.abs(got[1] - got[wps]).max() <= 1e-6 * scale
        for bad, err in ((wmax + 1, "MOFF_ERR_UNSUPPORTED"), (0, "MOFF_ERR_INVALID_ARG")):
            with pytest.raises(moff.MoffError, match=err):
                p.set_adjoint_waves(bad)
        p.autotune(E, g)
        assert 1 <= p.adjoint_waves()[0] <= wmax
        tuned = p.gain_vjp(E, g, Rd).cpu().numpy().astype(np.complex128)
        assert rel_err(tuned, ref) <= TOL
    small_plan = synth.make_config(1)
    with moff.Plan.from_geometry(small_plan.geom, device=0) as p:
        assert p.adjoint_waves() == (1, 1)
        with pytest.raises(moff.MoffError, match="MOFF_ERR_UNSUPPORTED"):
            p.set_adjoint_waves(2)
