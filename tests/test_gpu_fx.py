"""GPU visibility route (moff_image_fx) through the C ABI.

Sec. 2 of the paper shows that the MOFF image equals the image made from
visibilities (eq. dirty-image-FX through eq. e-field-conv).  The device FX route
correlates antenna pairs, grids each visibility with the pair's table response
and transforms the lag grid once; it shares no kernel with the MOFF path.  It is
checked against the FP64 oracle's FX route (`oracle.fx_discrete_image`) and
against the device MOFF image, with the float32 tolerance of the MOFF parity
tests: per channel, relative to Pbar = S / T (the mean squared field before
self-power removal),
    err_inf = max |I - I_ref| / max |Pbar| <= 1e-5,  err_2 = ||I - I_ref|| / ||Pbar|| <= 1e-5.
"""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import (CASES, TOL, _replay_matches, assert_image_close, moff, oracle_channels,  # noqa: F401
                             to_dev, torch)

pytestmark = pytest.mark.gpu


def run_fx(torch, moff, w, extra_flags=0):
    with moff.Plan.from_geometry(w.geom, device=0, extra_flags=extra_flags) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains) if w.gains is not None else None
        out = p.image_fx(E, g)
        torch.cuda.synchronize()
        return out.cpu().numpy()


# 4+4-bit samples over two 64-antenna correlator tiles (the second ragged) and
# 70 samples (one full 64-sample step and a ragged one), two table types
FX_CASES = dict(CASES, hetero_n100_ci4_t70=lambda: synth.random_case(
    25, 100, 64, 2, 70, [synth.random_kernel(np.random.default_rng(8), 3), synth.random_kernel(np.random.default_rng(9), 2)],
    fmt=synth.IN_CI4, extent_m=40.0, cell_m=1.5))


@pytest.mark.parametrize("case", ["config1", "config2_sub", "config5_sub", "hetero_n8", "hetero_n16",
                                  "hetero_n32_ci4", "hetero_n128_4types", "hetero_n100_ci4_t70"])
def test_fx_route_matches_oracle_fx(torch, moff, case):
    """Device FX image against the oracle's FX route (zero spacings left out):
    one to four table types of different sizes (the binning and the lag grid
    are formed for half the cells and mirrored across type pairs (p, q) and
    (q, p)), 4+4-bit and complex64 samples, gains, grids 8-256, antenna counts
    that leave the last 64-wide correlator tile ragged, T not a multiple of the
    32-sample chunk or the 64-sample step."""
    w = FX_CASES[case]()
    C = w.geom.n_chan
    got = run_fx(torch, moff, w)
    assert np.isfinite(got).all()
    _, pbar = oracle_channels(w, range(C))
    ref = np.stack([oracle.fx_discrete_image(w.geom, w.E, w.gains, c) for c in range(C)])
    assert_image_close(got, ref, pbar, label=f"{case} FX")


@pytest.mark.parametrize("flag", ["autocorr_none", "norm_pairs"])
def test_fx_flags(torch, moff, flag):
    """Zero-spacing terms kept (MOFF_AUTOCORR_NONE) and pair normalisation."""
    w = synth.make_config(1, n_time=16)
    w.geom.flags |= synth.AUTOCORR_NONE if flag == "autocorr_none" else synth.NORM_PAIRS
    _, pbar = oracle_channels(w, [0])
    if flag == "norm_pairs":
        pbar = pbar / (16 * 15)
    ref = oracle.fx_discrete_image(w.geom, w.E, w.gains, 0)[None]
    got = run_fx(torch, moff, w)
    assert_image_close(got, ref, pbar, label=f"FX {flag}")


@pytest.mark.parametrize("shape", [("config2", 200, 16), ("config3", 8, 4), ("config5", 1, 2), ("config5", 1, 256)])
def test_fx_route_equals_device_moff_image(torch, moff, shape):
    """Cross-method check on the device at sizes the oracle would take long for:
    the FX image equals moff_image (LWA-shaped 256 antennas; HERA-shaped 350
    antennas with 7x7 tables on the 256 grid; the 1024-antenna two-type
    calibration layout with one time sample; over all 256 channels its
    workspace of about 10.6 MB per channel runs in two chunks).  Pbar comes from
    the device MOFF image without self-power removal."""
    cfg, T, C = shape
    w = synth.make_config(int(cfg[-1]), n_time=T, n_chan=C)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains) if w.gains is not None else None
        img = p.image(E, g)
        fx = p.image_fx(E, g)
        torch.cuda.synchronize()
        img, fx = img.cpu().numpy(), fx.cpu().numpy()
    w.geom.flags |= synth.AUTOCORR_NONE
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        pbar = p.image(to_dev(torch, w.E), to_dev(torch, w.gains) if w.gains is not None else None)
        torch.cuda.synchronize()
        pbar = pbar.cpu().numpy().astype(np.float64)
    assert np.isfinite(fx).all()
    assert_image_close(fx, img.astype(np.float64), pbar, label=f"{cfg} FX vs MOFF")


def test_fx_rejects_bad_arguments(torch, moff):
    w = synth.make_config(1, n_time=4)
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        with pytest.raises(moff.MoffError):
            p.image_fx(E[:0])


@pytest.mark.parametrize("case", ["config2_sub", "config5_sub"])
def test_fx_deterministic_and_graph_replay(torch, moff, case):
    """Fixed-order sums: two eager calls agree bitwise, and the route captured in
    a HIP graph (after the first call has built its tables and workspace)
    reproduces the eager image on every replay (4+4-bit: int8 matrix-core
    correlator; complex64: float32 correlator)."""
    w = CASES[case]()
    C, N = w.geom.n_chan, w.geom.grid_n
    with moff.Plan.from_geometry(w.geom, device=0) as p:
        E = to_dev(torch, w.E)
        g = to_dev(torch, w.gains) if w.gains is not None else None
        first = p.image_fx(E, g).clone()
        out = torch.empty((C, N, N), dtype=torch.float32, device="cuda:0")
        eager = _replay_matches(torch, lambda st: p.image_fx(E, g, out=out, stream=st), out)
        assert torch.equal(first, eager)
