"""moff_image_noalloc (the entry point for callers that cannot allocate)
against moff_image through the C ABI, and against the FP64 oracle.

Two calls in a row on one plan, the second with a smaller input, each with a
launch configuration whose scratch holds per-slice partial sums; the first
also holds float64 running sums (slices longer than 256 samples).  The same
launch configuration gives the same kernels and summation order, so the two
entry points must agree bitwise; both must meet the 1e-5 parity bar of the
other GPU tests.  A request whose scratch cannot fit is rejected before any
launch.
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
    m._lib.lib()
    return m


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check_oracle(w, got, T):
    P = oracle.plan(w.geom)
    for c in range(w.geom.n_chan):
        ref, parts = oracle.moff_channel(w.geom, w.E[:T], w.gains, c, P, keep=True)
        pbar = parts["S"] / T
        d = got[c].astype(np.float64) - ref
        e_inf = np.abs(d).max() / np.abs(pbar).max()
        e_2 = np.linalg.norm(d) / np.linalg.norm(pbar)
        assert e_inf <= TOL and e_2 <= TOL, (c, e_inf, e_2)


def test_noalloc_matches_image_two_calls(torch, moff):
    w = synth.make_config(2, n_time=600, n_chan=4)
    print("noalloc: config-2 subset, 4 channels, T = 600 then 400, 2 slices", flush=True)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        p.set_config(0, 2)
        E = to_dev(torch, w.E)
        for T in (600, 400):           # the second call smaller: 200 samples per slice
            Et = E[:T].contiguous()
            ref_dev = p.image(Et)
            out = torch.full_like(ref_dev, float("nan"))
            torch.cuda.synchronize()
            p.image_noalloc(Et, out=out)
            torch.cuda.synchronize()
            got, ref = out.cpu().numpy(), ref_dev.cpu().numpy()
            assert np.array_equal(got, ref), f"T={T}: max diff {np.abs(got - ref).max()}"
            check_oracle(w, got, T)


def test_noalloc_gains_and_one_slice(torch, moff):
    w = synth.make_config(5, n_time=6, n_chan=2)
    print("noalloc: calibration layout, 2 channels, T = 6 then 4, gains, 3 slices then 2", flush=True)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains)
        for T, sl in ((6, 3), (4, 2)):
            p.set_config(1, sl)
            Et = E[:T].contiguous()
            ref = p.image(Et, gains=g)
            out = torch.full_like(ref, float("nan"))
            p.image_noalloc(Et, gains=g, out=out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            check_oracle(w, out.cpu().numpy(), T)


def test_noalloc_rejects_oversized_scratch(torch, moff):
    # 300 channels of a 256 grid with 257 samples in one slice need
    # 8 * 300 * 256^2 bytes of float64 running sums: more than the fixed array
    w = synth.make_config(3, n_time=2, n_chan=300)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        p.set_config(1, 1)
        E = torch.zeros((257, 300, w.geom.n_ant), dtype=torch.uint8, device="cuda:0")
        out = torch.empty((300, 256, 256), dtype=torch.float32, device="cuda:0")
        with pytest.raises(moff.MoffError) as ei:
            p.image_noalloc(E, out=out)
        assert ei.value.status == 4
