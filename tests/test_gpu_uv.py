"""GPU: the uv-plane autocorrelation rule (MOFF_AUTOCORR_UV, Sec. 4.2) against
the FP64 oracle, which takes the paper's steps literally (to the uv plane,
subtract the scaled autocorrelation kernel at zero spacing, back to the image).
FP32 paths: err_inf, err_2 <= 1e-5 relative to the oracle's mean squared field,
as for the exact removal; the reduced-precision path keeps its stated 16u / 4u.
The gradient under the rule is checked against central differences of the
oracle's uv image."""
import numpy as np
import pytest

import oracle
import synth
from oracle import uv_autocorr

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
    m._lib.lib()
    return m


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def oracle_uv(w, channels):
    """Oracle images and the error metric's reference scale Pbar = S / T, with
    the image's pair normalisation 1 / (N_a (N_a - 1)) when that flag is set."""
    P = oracle.plan(w.geom)
    na = w.geom.n_ant
    norm = 1.0 / (na * (na - 1)) if int(w.geom.flags) & synth.NORM_PAIRS else 1.0
    imgs, pbars = [], []
    for c in channels:
        img, parts = uv_autocorr.uv_channel(w.geom, w.E, w.gains, c, P, keep=True)
        imgs.append(img)
        pbars.append(parts["Pbar"] * norm)
    return np.stack(imgs), np.stack(pbars)


def assert_close(got, ref, pbar, tol, label, tol_2=None):
    tol_2 = tol if tol_2 is None else tol_2
    for c in range(ref.shape[0]):
        d = got[c].astype(np.float64) - ref[c]
        ei = np.abs(d).max() / np.abs(pbar[c]).max()
        e2 = np.linalg.norm(d) / np.linalg.norm(pbar[c])
        assert ei <= tol and e2 <= tol_2, f"{label} channel {c}: err_inf={ei:.3g} err_2={e2:.3g}"


def run(torch, moff, w, how="image", extra=0):
    flags = synth.AUTOCORR_UV | extra
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=flags) as p:
        E = dev(torch, w.E)
        g = dev(torch, w.gains) if w.gains is not None else None
        if how == "image":
            out = p.image(E, g)
        elif how == "staged":
            out = p.image_staged(E, g)
        else:
            import torch as t
            C, N = w.geom.n_chan, w.geom.grid_n
            S = t.zeros((C, N, N), dtype=t.float32, device="cuda:0")
            A = t.zeros((C, w.geom.n_ktypes), dtype=t.float64, device="cuda:0")
            T = w.E.shape[0]
            p.accumulate(E[: T // 2], S, A, g)
            p.accumulate(E[T // 2:], S, A, g)
            out = p.finalize(S, A, T)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def _lattice(seed=4):
    rng = np.random.default_rng(seed)
    g = np.arange(6, dtype=np.float64) * 3.0
    xy = np.stack(np.meshgrid(g, g), -1).reshape(-1, 2) + 0.25
    geom = synth.Geometry(ant_xy=xy, ktype_k=[2], ktype_vals=[synth.random_kernel(rng, 2)],
                          ant_ktype=np.zeros(len(xy), np.int32), freq_hz=np.array([60e6, 70e6]), grid_n=64,
                          cell_m=1.0, flags=synth.IN_C64)
    E = (rng.standard_normal((5, 2, len(xy))) + 1j * rng.standard_normal((5, 2, len(xy)))).astype(np.complex64)
    return synth.Workload(name="lattice", geom=geom, E=E, gains=synth.random_gains(rng, 2, len(xy)), n_time=5)


def _hetero(flags=0):
    rng = np.random.default_rng(12)
    w = synth.random_case(33, 30, 64, 2, 4, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 5)],
                          extent_m=20.0, cell_m=1.0)
    w.geom.flags |= flags
    return w


CASES = {
    "config1": lambda: synth.make_config(1),
    "config2_sub": lambda: synth.make_config(2, n_time=6, n_chan=2),
    "config5_sub": lambda: synth.make_config(5, n_time=3, n_chan=2),
    "hetero_pairs": lambda: _hetero(synth.NORM_PAIRS),
    "lattice_no_overlap": _lattice,
}


@pytest.mark.parametrize("case", list(CASES))
def test_uv_image_vs_oracle(torch, moff, case):
    w = CASES[case]()
    ref, pbar = oracle_uv(w, range(w.geom.n_chan))
    got = run(torch, moff, w)
    assert_close(got, ref, pbar, TOL, case)
    if case == "lattice_no_overlap":   # no overlapping footprints: the rule is the exact removal
        with moff.Plan.from_geometry(w.geom, device=0) as p:
            exact = p.image(dev(torch, w.E), dev(torch, w.gains))
            torch.cuda.synchronize()
        assert_close(exact.cpu().numpy(), ref, pbar, TOL, "exact removal")


@pytest.mark.parametrize("how", ["staged", "split"])
def test_uv_staged_and_split_accumulation(torch, moff, how):
    w = CASES["config5_sub"]()
    ref, pbar = oracle_uv(w, range(w.geom.n_chan))
    assert_close(run(torch, moff, w, how), ref, pbar, TOL, how)


def test_uv_reduced_precision(torch, moff):
    w = synth.make_config(4, n_time=6, n_chan=2, grid_n=64)
    ref, pbar = oracle_uv(w, range(2))
    u = 2.0 ** -11
    assert_close(run(torch, moff, w, extra=synth.MFMA_F16), ref, pbar, 16 * u, "mfma f16", tol_2=4 * u)


def test_uv_gradient_vs_finite_differences(torch, moff):
    rng = np.random.default_rng(17)
    w = synth.random_case(18, 10, 32, 2, 3, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 2)],
                          extent_m=8.0, cell_m=1.0)
    model = rng.standard_normal((2, 32, 32)) * 3.0

    def loss(g):
        img = uv_autocorr.uv_image(w.geom, w.E, g)
        return float(np.sum((img - model) ** 2)), 2.0 * (img - model)

    g0 = w.gains.astype(np.complex128)
    _, R = loss(g0)
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=synth.AUTOCORR_UV) as p:
        got = p.gain_vjp(dev(torch, w.E), dev(torch, w.gains), dev(torch, R.astype(np.float32)))
        torch.cuda.synchronize()
        got = got.cpu().numpy().astype(np.complex128)
    h = 1e-6
    for _ in range(6):
        d = rng.standard_normal(g0.shape) + 1j * rng.standard_normal(g0.shape)
        fd = (loss(g0 + h * d)[0] - loss(g0 - h * d)[0]) / (2 * h)
        an = float(np.real(np.sum(np.conj(got) * d)))
        assert abs(fd - an) <= 1e-4 * np.sum(np.abs(got) * np.abs(d)), (fd, an)
