"""Device images against the hand-derived golden fixtures of
`tests/golden/two_antenna_fringes.txt` (N = 8, T = 1, unit gains; see the
file's header for the derivations from Sec. 2, Sec. 3 and Sec. 4.2).  These fix
the exponent sign, the image axes, the table orientation, the unnormalised
transform and the self-power removal without going through the oracle.  Each
case runs through the fused kernel, the staged pipeline and the visibility
(FX) route; float32 arithmetic on values of order 1-9, compared to 1e-5.

The library takes at least two antennas, so the single-antenna cases D-F get
a second antenna at cell (2, 2) with zero field: its pair terms and its self
power vanish, and the hand-derived values hold unchanged."""
import os

import numpy as np
import pytest

import synth
from test_gpu_parity import moff, to_dev, torch  # noqa: F401

pytestmark = pytest.mark.gpu

ONE = np.ones((1, 1))
CASES = {
    "A": ([[0, 0], [1, 0]], ONE, [1, 1], 0),
    "B": ([[0, 0], [1, 0]], ONE, [1, 1j], 0),
    "C": ([[0, 0], [0, 1]], ONE, [1, 1j], 0),
    "D": ([[0, 0], [2, 2]], np.array([[1, 2], [0, 0]]), [1, 0], synth.AUTOCORR_NONE),
    "E": ([[0, 0], [2, 2]], np.array([[1, 0], [1j, 0]]), [1, 0], synth.AUTOCORR_NONE),
    "F": ([[0, 0], [2, 2]], np.array([[1, 2], [0, 0]]), [1, 0], 0),
}


def golden_rows(golden_dir):
    rows = {}
    with open(os.path.join(golden_dir, "two_antenna_fringes.txt")) as f:
        for line in f:
            s = line.strip()
            if s and not s.startswith("#"):
                name, axis, *vals = s.split()
                rows[name] = (axis, np.asarray([float(v) for v in vals]))
    return rows


@pytest.mark.parametrize("path", ["fused", "staged", "fx"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_device_images_match_golden(torch, moff, golden_dir, name, path):
    cells_xy, kernel, e, flags = CASES[name]
    geom = synth.Geometry(ant_xy=np.asarray(cells_xy, np.float64), ktype_k=[kernel.shape[0]],
                          ktype_vals=[kernel.astype(np.complex64)], ant_ktype=np.zeros(len(cells_xy), np.int32),
                          freq_hz=np.array([50e6]), grid_n=8, cell_m=1.0, flags=synth.IN_C64 | flags)
    E = np.asarray(e, np.complex64).reshape(1, 1, -1)
    axis, want = golden_rows(golden_dir)[name]
    with moff.Plan.from_geometry(geom, device=0) as p:
        Ed = to_dev(torch, E)
        out = {"fused": p.image, "staged": p.image_staged, "fx": p.image_fx}[path](Ed)
        torch.cuda.synchronize()
        img = out.cpu().numpy()[0].astype(np.float64)
    prof = img if axis == "r" else img.T      # prof[j, other] varies with j
    for j in range(8):
        assert np.allclose(prof[j], want[j], atol=1e-5), (name, path, j, prof[j], want[j])
