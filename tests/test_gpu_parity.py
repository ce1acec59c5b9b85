"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance (FP32 path): per channel, with Pbar = S / T the oracle's mean squared
field before self-power removal,
    err_inf = max |I_gpu - I_oracle| / max |Pbar|  <= 1e-5
    err_2   = ||I_gpu - I_oracle||_2 / ||Pbar||_2  <= 1e-5
Per-pixel relative error is not used: removing the self power cancels most of
|Y|^2 at pixels without sky signal.  Cell indices are compared bit-exactly by
the host tests.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


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
    P = oracle.plan(w.geom)
    imgs, pbar = [], []
    for c in channels:
        img, parts = oracle.moff_channel(w.geom, w.E, w.gains, c, P, keep=True)
        imgs.append(img)
        pbar.append(parts["S"] / w.E.shape[0])
    return np.stack(imgs), np.stack(pbar)


def assert_image_close(got, ref, pbar, tol=TOL, label=""):
    for c in range(ref.shape[0]):
        d = got[c].astype(np.float64) - ref[c]
        e_inf = np.abs(d).max() / np.abs(pbar[c]).max()
        e_2 = np.linalg.norm(d) / np.linalg.norm(pbar[c])
        assert e_inf <= tol and e_2 <= tol, f"{label} channel {c}: err_inf={e_inf:.3g} err_2={e_2:.3g}"


def run_image(torch, moff, w, staged=False):
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains) if w.gains is not None else None
        out = p.image_staged(E, g) if staged else p.image(E, g)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def _zero_corners(seed, k):
    K = synth.random_kernel(np.random.default_rng(seed), k).copy()
    K[0, 0] = K[0, -1] = K[-1, 0] = K[-1, -1] = 0
    return K


CASES = {
    "config1": lambda: synth.make_config(1),
    "config2_sub": lambda: synth.make_config(2, n_time=7, n_chan=3),
    "config3_sub": lambda: synth.make_config(3, n_time=3, n_chan=2),
    "config4_n64": lambda: synth.make_config(4, n_time=5, n_chan=2, grid_n=64),
    "config5_sub": lambda: synth.make_config(5, n_time=3, n_chan=2),
    "hetero_n8": lambda: synth.random_case(21, 5, 8, 2, 3, [synth.random_kernel(np.random.default_rng(1), 2)],
                                           extent_m=1.5, cell_m=1.0),
    "hetero_n16": lambda: synth.random_case(22, 9, 16, 2, 5, [synth.random_kernel(np.random.default_rng(2), 3),
                                                              synth.random_kernel(np.random.default_rng(3), 2)],
                                            extent_m=4.0, cell_m=1.0),
    "hetero_n32_ci4": lambda: synth.random_case(23, 20, 32, 3, 4, [synth.random_kernel(np.random.default_rng(4), 3),
                                                                   synth.random_kernel(np.random.default_rng(5), 4)],
                                                fmt=synth.IN_CI4, extent_m=20.0, cell_m=1.5),
    # complex tables with exactly-zero corners at N = 256: the gather leaves the
    # zero entries out, and the 512-thread shape's program is wave-owned
    # (each wave grids the rows it transforms) with complex weights
    "hetero_n256_zero_taps": lambda: synth.random_case(25, 220, 256, 2, 3, [_zero_corners(9, 5), _zero_corners(10, 7)],
                                                       extent_m=120.0, cell_m=1.0),
    "hetero_n128_4types": lambda: synth.random_case(24, 150, 128, 2, 3,
                                                    [synth.random_kernel(np.random.default_rng(6 + i), k)
                                                     for i, k in enumerate((1, 3, 5, 7))],
                                                    extent_m=90.0, cell_m=1.6),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fused_image_parity(torch, moff, case):
    w = CASES[case]()
    ref, pbar = oracle_channels(w, range(w.geom.n_chan))
    got = run_image(torch, moff, w)
    assert_image_close(got, ref, pbar, label=case)


@pytest.mark.parametrize("case", ["config1", "config2_sub", "config5_sub", "hetero_n16"])
def test_staged_image_parity(torch, moff, case):
    w = CASES[case]()
    ref, pbar = oracle_channels(w, range(w.geom.n_chan))
    got = run_image(torch, moff, w, staged=True)
    assert_image_close(got, ref, pbar, label=case)


@pytest.mark.parametrize("case", ["config1", "config2_sub", "hetero_n32_ci4", "config5_sub"])
def test_grid_parity(torch, moff, case):
    w = CASES[case]()
    P = oracle.plan(w.geom)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        eg = p.grid(to_dev(torch, w.E), to_dev(torch, w.gains) if w.gains is not None else None)
        A = torch.zeros((w.geom.n_chan, w.geom.n_ktypes), dtype=torch.float64, device="cuda:0")
        p.self_power(to_dev(torch, w.E), A, to_dev(torch, w.gains) if w.gains is not None else None)
        torch.cuda.synchronize()
        eg = eg.cpu().numpy()
        A = A.cpu().numpy()
    for c in range(w.geom.n_chan):
        e = oracle.calibrated_field(w.E, w.gains, w.geom.flags, c)
        ref = oracle.grid_field(e, P)
        scale = np.abs(ref).max()
        assert np.abs(eg[:, c] - ref).max() <= 1e-6 * scale
        refA = oracle.self_power(e, P["ant_ktype"], P["n_types"])
        assert np.allclose(A[c], refA, rtol=1e-6)     # e = g E is formed in float32, |e|^2 summed in float64


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 256])
def test_fft2_parity(torch, moff, N):
    rng = np.random.default_rng(N)
    L = N // 2
    w = synth.random_case(30 + N, 3, N, 1, 1, [np.ones((1, 1), np.complex64)], extent_m=1.0, cell_m=1.0)
    F = 5
    Eg = (rng.standard_normal((F, L, L)) + 1j * rng.standard_normal((F, L, L))).astype(np.complex64)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        Y = p.fft2(to_dev(torch, Eg))
        torch.cuda.synchronize()
        Y = Y.cpu().numpy()
    ref = oracle.image_field(Eg.astype(np.complex128), N)
    for f in range(F):
        err = np.abs(Y[f] - ref[f]).max() / np.abs(ref[f]).max()
        assert err <= 2e-6, (N, f, err)


def test_detect_accumulate_and_finalize(torch, moff):
    w = CASES["config2_sub"]()
    ref, pbar = oracle_channels(w, range(w.geom.n_chan))
    P = oracle.plan(w.geom)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        Y = p.fft2(p.grid(E))
        S = torch.zeros((3, 128, 128), dtype=torch.float32, device="cuda:0")
        A = torch.zeros((3, 1), dtype=torch.float64, device="cuda:0")
        p.detect_accumulate(Y, S)
        p.self_power(E, A)
        img = p.finalize(S, A, w.E.shape[0])
        torch.cuda.synchronize()
        S = S.cpu().numpy()
        img = img.cpu().numpy()
    for c in range(3):
        assert np.abs(S[c] / w.E.shape[0] - pbar[c]).max() <= 1e-5 * np.abs(pbar[c]).max()
    assert_image_close(img, ref, pbar, label="staged by hand")


def test_accumulate_split_equals_whole(torch, moff):
    w = synth.make_config(2, n_time=12, n_chan=2)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        S = torch.zeros((2, 128, 128), dtype=torch.float32, device="cuda:0")
        A = torch.zeros((2, 1), dtype=torch.float64, device="cuda:0")
        p.accumulate(E[:5].contiguous(), S, A)
        p.accumulate(E[5:].contiguous(), S, A)
        split = p.finalize(S, A, 12)
        whole = p.image(E)
        torch.cuda.synchronize()
        split, whole = split.cpu().numpy(), whole.cpu().numpy()
    ref, pbar = oracle_channels(w, range(2))
    assert_image_close(split, ref, pbar, label="split")
    assert_image_close(whole, ref, pbar, label="whole")


def test_long_integration_one_slice(torch, moff):
    """A long integration in one time slice (Sec. 3 time averaging): 100,000
    samples summed by a single workgroup per column class.  The float32
    register sums are folded into float64 every 256 samples, so the
    accumulation adds well under 1e-6 here (2e-8 in a CPU simulation of that
    summation order); one float32 sum over all samples would add about 9e-6
    on this input (the same simulation).  The oracle runs over time chunks and sums S and A,
    which are linear in the frames."""
    T, chunk = 100_000, 5_000
    w = synth.make_config(1, n_time=T)
    print(f"long integration: config 1, T = {T}, one slice", flush=True)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        p.set_config(0, 1)
        assert p.config(T)["slices"] == 1
        got = p.image(to_dev(torch, w.E))
        torch.cuda.synchronize()
        got = got.cpu().numpy()[0].astype(np.float64)
    P = oracle.plan(w.geom)
    S, A = 0.0, 0.0
    for t0 in range(0, T, chunk):
        _, parts = oracle.moff_channel(w.geom, w.E[t0:t0 + chunk], w.gains, 0, P, keep=True)
        S, A = S + parts["S"], A + parts["A"]
    ref = (S - np.tensordot(A, parts["P"], axes=1)) / T
    pbar = S / T
    e_inf = np.abs(got - ref).max() / np.abs(pbar).max()
    e_2 = np.linalg.norm(got - ref) / np.linalg.norm(pbar)
    assert e_inf <= TOL and e_2 <= TOL, (e_inf, e_2)
    assert e_inf <= 2e-6, f"accumulation error {e_inf:.3g}: float32 sums are not blocked"


@pytest.mark.parametrize("N", [8, 16])
def test_blocked_accumulation_small_grids(torch, moff, N):
    """Grids whose workgroups have lanes without a column (the running sums
    hold more values than pixels): 600 samples in one slice, so the float32
    sums are folded into the float64 running sums twice."""
    rng = np.random.default_rng(N)
    w = synth.random_case(N, 5, N, 2, 600, [synth.random_kernel(rng, 2)], extent_m=N / 6.0, cell_m=1.0)
    ref, pbar = oracle_channels(w, range(2))
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        p.set_config(0, 1)
        got = p.image(to_dev(torch, w.E), gains=to_dev(torch, w.gains))
        torch.cuda.synchronize()
        got = got.cpu().numpy()
    assert_image_close(got, ref, pbar, label=f"N={N} blocked")


def test_finalize_long_integration_count(torch, moff):
    """moff_finalize only scales and subtracts: a total sample count beyond
    2^31 / n_chan (a long streamed integration) is accepted and gives
    (S - sum_p A_p P_p) / T from the streamed sums."""
    w = synth.make_config(5, n_time=3, n_chan=2)
    T_total = (1 << 31) // w.geom.n_chan + 1
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        S = torch.zeros((2, 256, 256), dtype=torch.float32, device="cuda:0")
        A = torch.zeros((2, 2), dtype=torch.float64, device="cuda:0")
        p.accumulate(E, S, A, gains=to_dev(torch, w.gains))
        img = p.finalize(S, A, T_total)
        torch.cuda.synchronize()
        S, A, img = S.cpu().numpy().astype(np.float64), A.cpu().numpy(), img.cpu().numpy()
        Pp = np.stack([p.power_pattern(k) for k in range(2)])
    ref = (S - np.einsum("cp,pij->cij", A, Pp)) / T_total
    scale = np.abs(S).max() / T_total
    assert np.abs(img - ref).max() <= 1e-6 * scale


@pytest.mark.parametrize("flag", ["autocorr_none", "norm_pairs"])
def test_flags(torch, moff, flag):
    w = synth.make_config(1, n_time=16)
    w.geom.flags |= synth.AUTOCORR_NONE if flag == "autocorr_none" else synth.NORM_PAIRS
    ref, pbar = oracle_channels(w, [0])
    got = run_image(torch, moff, w)
    if flag == "norm_pairs":
        pbar = pbar / (16 * 15)
    assert_image_close(got, ref, pbar, label=flag)


def test_flagged_antenna_and_single_sample(torch, moff):
    w = synth.make_config(5, n_time=1, n_chan=2)
    w.gains[:, 17] = 0
    w.gains[1, 500:520] = 0
    ref, pbar = oracle_channels(w, range(2))
    got = run_image(torch, moff, w)
    assert_image_close(got, ref, pbar, label="flags")


def test_deterministic(torch, moff):
    w = synth.make_config(2, n_time=9, n_chan=4)
    a = run_image(torch, moff, w)
    b = run_image(torch, moff, w)
    assert np.array_equal(a, b)


def test_full_config2_sampled_channels(torch, moff):
    """The benchmark workload at full size and in the benchmark's launch
    configuration, checked on channels the oracle computes one by one."""
    w = synth.make_config(2)
    got = run_image(torch, moff, w)
    assert np.isfinite(got).all()
    chans = [0, 77, 127]
    ref, pbar = oracle_channels(w, chans)
    assert_image_close(got[chans], ref, pbar, label="config2 full")


@pytest.mark.parametrize("case", ["config2_sub", "config3_sub", "config5_sub", "hetero_n128_4types",
                                  "hetero_n256_zero_taps", "config1"])
def test_every_variant_and_slicing(torch, moff, case):
    """Every shape variant of the frame transform and several time slicings agree
    with the oracle (the autotuner may pick any of them)."""
    w = CASES[case]()
    ref, pbar = oracle_channels(w, range(w.geom.n_chan))
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains) if w.gains is not None else None
        nvar = p.config(w.E.shape[0])["n_variants"]
        for v in range(nvar):
            for sl in (1, 2, 3):
                p.set_config(variant=v, slices=sl)
                cfg = p.config(w.E.shape[0])
                assert cfg["variant"] == v and cfg["slices"] == min(sl, w.E.shape[0])
                got = p.image(E, g)
                torch.cuda.synchronize()
                assert_image_close(got.cpu().numpy(), ref, pbar, label=f"{case} v{v} s{sl}")


@pytest.mark.parametrize("n_ant,grid_n", [(128, 64), (129, 64), (256, 128), (257, 128)])
def test_antennas_per_lane_boundary(torch, moff, n_ant, grid_n):
    """Up to one antenna per lane (n_ant no larger than the workgroup: 128
    threads at N = 64, 256 at N = 128) and one more: the two kernel instances
    keep each antenna type's self power differently (one sum per lane, typed
    after the frame loop, or one running sum per type), and both images agree
    with the oracle, for every shape variant, with three table types."""
    kernels = [synth.random_kernel(np.random.default_rng(30 + i), k) for i, k in enumerate((1, 3, 5))]
    w = synth.random_case(40 + n_ant, n_ant, grid_n, 2, 3, kernels, extent_m=grid_n * 0.35, cell_m=1.0)
    ref, pbar = oracle_channels(w, range(w.geom.n_chan))
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains)
        for v in range(p.config(w.E.shape[0])["n_variants"]):
            p.set_config(variant=v, slices=1)
            got = p.image(E, g)
            torch.cuda.synchronize()
            assert_image_close(got.cpu().numpy(), ref, pbar, label=f"n_ant {n_ant} v{v}")


def test_autotune_and_graph_replay(torch, moff):
    """The autotuned configuration is correct, and the fused call captured in a
    HIP graph reproduces the eager result on every replay."""
    w = synth.make_config(2, n_time=20, n_chan=6)
    ref, pbar = oracle_channels(w, range(6))
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        cfg = p.autotune(E)
        assert cfg["tuned"] == 1
        out = torch.empty((6, 128, 128), dtype=torch.float32, device="cuda:0")
        p.image(E, out=out)                     # allocates the workspace before capture
        torch.cuda.synchronize()
        eager = out.clone()
        assert_image_close(eager.cpu().numpy(), ref, pbar, label="autotuned")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                p.image(E, out=out, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(3):
            out.fill_(-1.0)                     # eager work between replays
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"replay {rep} differs"


@pytest.mark.parametrize("cfg,chans", [(3, [0, 511, 1023]), (5, [0, 255])])
def test_full_size_sampled_channels(torch, moff, cfg, chans):
    """HERA-shaped and calibration workloads at full size (every channel imaged in
    one launch, autotuned), checked on channels the oracle computes one by one.
    The same autotuned launch captured in a HIP graph gives the eager result
    bitwise on three replays, with eager work between them."""
    w = synth.make_config(cfg)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains) if w.gains is not None else None
        p.autotune(E, g)
        out = p.image(E, g)                     # also sizes the workspace before capture
        torch.cuda.synchronize()
        eager = out.clone()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                p.image(E, g, out=out, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(3):
            out.fill_(float("nan"))             # eager work between replays
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"config {cfg}: graph replay {rep} differs from the eager call"
        got = eager.cpu().numpy()
        del graph
    assert np.isfinite(got).all()
    ref, pbar = oracle_channels(w, chans)
    assert_image_close(got[chans], ref, pbar, label=f"config{cfg} full")


@pytest.mark.parametrize("case", ["config1", "config2_sub", "config5_sub", "hetero_n32_ci4"])
def test_fused_image_equals_visibility_route(torch, moff, case):
    """Cross-method check of the device output (Sec. 2: the MOFF image equals the
    visibility-based image, eq. dirty-image-FX, through eq. e-field-conv): the GPU
    MOFF image against the oracle's FX route, which correlates antenna pairs,
    grids each visibility with the cross-correlation of the two placed footprints
    and transforms once, sharing no step with the MOFF oracle."""
    w = CASES[case]()
    got = run_image(torch, moff, w)
    _, pbar = oracle_channels(w, range(w.geom.n_chan))
    fx = np.stack([oracle.fx_discrete_image(w.geom, w.E, w.gains, c) for c in range(w.geom.n_chan)])
    assert_image_close(got, fx, pbar, label=f"{case} vs FX route")


def _replay_matches(torch, call, out):
    """Capture `call(stream)` (which writes `out`) in a graph after one eager call,
    then replay it three times with eager work and synchronisation in between;
    every replay must reproduce the eager result exactly."""
    call(torch.cuda.current_stream())          # allocates any workspace before capture
    torch.cuda.synchronize()
    eager = out.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            call(s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep} differs"
    return eager


@pytest.mark.parametrize("kind", ["mfma_f16", "uv_rule", "gain_adjoint"])
def test_graph_replay_other_paths(torch, moff, kind):
    """The matrix-core image, the uv-plane rule (zero fill, fused kernel, per-channel
    finalisation) and the fused gain adjoint (kernel, reductions, final pass)
    captured in HIP graphs: every replay equals the eager call."""
    if kind == "mfma_f16":
        w = synth.make_config(4, n_time=12, n_chan=3, grid_n=64)
        flags = synth.MFMA_F16
    elif kind == "uv_rule":
        w = synth.make_config(2, n_time=12, n_chan=3)
        flags = synth.AUTOCORR_UV
    else:
        w = synth.make_config(5, n_time=4, n_chan=2)
        flags = 0
    C, N = w.geom.n_chan, w.geom.grid_n
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=flags) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains) if w.gains is not None else None
        if kind == "gain_adjoint":
            R = torch.randn((C, N, N), dtype=torch.float32, device="cuda:0")
            out = torch.empty((C, w.geom.n_ant), dtype=torch.complex64, device="cuda:0")
            _replay_matches(torch, lambda st: p.gain_vjp(E, g, R, out=out, stream=st), out)
        else:
            out = torch.empty((C, N, N), dtype=torch.float32, device="cuda:0")
            _replay_matches(torch, lambda st: p.image(E, g, out=out, stream=st), out)
