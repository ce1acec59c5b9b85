"""GPU edge cases: the largest antenna count the plan accepts (4000) through every
path, the smallest array (2 antennas), and the C ABI's argument checks on a
device plan (no kernel runs for a rejected call)."""
import ctypes

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
    m._lib.lib()
    return m


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def close(got, w, channels, tol=TOL, tol_2=None):
    P = oracle.plan(w.geom)
    tol_2 = tol if tol_2 is None else tol_2
    for i, c in enumerate(channels):
        ref, parts = oracle.moff_channel(w.geom, w.E, w.gains, c, P, keep=True)
        pbar = parts["S"] / w.E.shape[0]
        d = got[i].astype(np.float64) - ref
        ei, e2 = np.abs(d).max() / np.abs(pbar).max(), np.linalg.norm(d) / np.linalg.norm(pbar)
        assert ei <= tol and e2 <= tol_2, (c, ei, e2)


def max_antennas(N, cell, n_ant=4000):
    rng = np.random.default_rng(40)
    return synth.random_case(41, n_ant, N, 2, 3, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 1)],
                             extent_m=(N // 2 - 4) * cell, cell_m=cell)


def test_max_antennas_fused_staged_tuned(torch, moff):
    w = max_antennas(256, 1.6)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E, g = dev(torch, w.E), dev(torch, w.gains)
        outs = [p.image(E, g), p.image_staged(E, g)]
        p.autotune(E, g)
        outs.append(p.image(E, g))
        torch.cuda.synchronize()
    for o in outs:
        close(o.cpu().numpy(), w, [0, 1])


@pytest.mark.parametrize("N,n_ant", [(64, 4000), (128, 1400)])
def test_max_antennas_reduced_precision(torch, moff, N, n_ant):
    """The matrix-core kernel double-buffers the samples, the grid and the
    transposed row-stage output in LDS: every count the plan accepts runs on
    the 64 grid, and on the 128 grid about 1490 antennas fit (these tables)."""
    w = max_antennas(N, 0.8 if N == 128 else 1.6, n_ant)
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=synth.MFMA_BF16) as p:
        got = p.image(dev(torch, w.E), dev(torch, w.gains))
        torch.cuda.synchronize()
    u = 2.0 ** -8
    close(got.cpu().numpy(), w, [0, 1], tol=16 * u, tol_2=4 * u)


def test_max_antennas_gradient(torch, moff):
    """4000 antennas exceed the fused adjoint's per-lane slots: the staged form runs."""
    w = max_antennas(64, 0.4)
    rng = np.random.default_rng(2)
    R = rng.standard_normal((2, 64, 64)).astype(np.float32)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        got = p.gain_vjp(dev(torch, w.E), dev(torch, w.gains), dev(torch, R))
        torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.complex128)
    ref = oracle.gain_gradient(w.geom, w.E, w.gains, R.astype(np.float64))
    err = max(np.abs(got[c] - ref[c]).max() / np.abs(ref[c]).max() for c in range(2))
    assert err <= 1e-4


def test_two_antennas(torch, moff):
    rng = np.random.default_rng(5)
    w = synth.random_case(6, 2, 8, 3, 4, [synth.random_kernel(rng, 2)], extent_m=2.0, cell_m=1.0)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        got = p.image(dev(torch, w.E), dev(torch, w.gains))
        torch.cuda.synchronize()
    close(got.cpu().numpy(), w, [0, 1, 2])


def test_c_abi_rejects_bad_arguments(torch, moff):
    from paper_1510_08318_amd import _lib
    w = synth.make_config(1, n_time=4)
    L = _lib.lib()
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = dev(torch, w.E)
        img = torch.empty((1, 32, 32), dtype=torch.float32, device="cuda:0")
        big = torch.empty(32 * 32 + 4, dtype=torch.float32, device="cuda:0")
        ok = L.moff_image(p.handle, E.data_ptr(), 4, None, img.data_ptr(), None)
        torch.cuda.synchronize()
        assert ok == 0
        assert L.moff_image(p.handle, E.data_ptr(), 0, None, img.data_ptr(), None) == 1        # no samples
        assert L.moff_image(p.handle, None, 4, None, img.data_ptr(), None) == 1                # null E
        assert L.moff_image(p.handle, E.data_ptr(), 4, None, None, None) == 1                  # null image
        assert L.moff_image(p.handle, E.data_ptr(), 4, None, big.data_ptr() + 4, None) == 1    # misaligned image
        assert L.moff_gain_vjp(p.handle, E.data_ptr(), 4, None, None, img.data_ptr(), None) == 1
        assert L.moff_plan_set_config(p.handle, 5, 0) == 1                                     # no such variant
        assert L.moff_plan_set_config(p.handle, 0, 300) == 1                                   # too many slices
        torch.cuda.synchronize()
