"""FP64 CPU oracle for the MOFF imaging path: TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library (`paper_1510_08318_amd`)
and neither imports the other; both consume the seeded inputs of `synth`.

Modules
  moff  the MOFF route: mapping, calibration, gridding, direct DFT, squaring,
        time averaging, per-antenna self-power removal.
  fx    the visibility (FX) routes used to pin `moff`: discrete footprints
        (exact identity) and analytic top-hat footprints (gridding coarseness).
  grad  the gradient of an image loss with respect to the complex gains.

Parity status: every function here is pinned by the CPU tests in
tests/test_oracle_pins.py (brute-force pair sums, the FX identity, Parseval,
library DFT, point-source closed form, hand-derived golden values, invariants)
and tests/test_oracle_grad.py (finite differences of the forward image, gauge
invariance, zero gradient at the true calibration).
"""
from .moff import (AUTOCORR_NONE, IN_C64, IN_CI4, NORM_PAIRS, FootprintOverflow,  # noqa: F401
                   calibrated_field, cell_indices, decode_ci4, default_cell_size,
                   dft_matrix, grid_field, image_field, image_field_literal,
                   moff_channel, moff_image, plan, power_pattern, self_power)
from .fx import fx_analytic_image, fx_discrete_image, visibilities  # noqa: F401
from .grad import gain_gradient, image_loss  # noqa: F401
from .uv_autocorr import uv_channel, uv_image  # noqa: F401
