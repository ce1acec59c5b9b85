"""Pins for the FP64 gain gradient: finite differences of the oracle's forward
image, the gauge (global phase) invariance of the image, and a zero gradient at
the calibration that reproduces the model sky (Sec. 3, calibration applied
before gridding)."""
import numpy as np
import pytest

import oracle
import synth


def _case(seed, flags=0, fmt=synth.IN_C64, N=16, n_ant=6, C=2, T=3):
    rng = np.random.default_rng(50 + seed)
    kern = [synth.random_kernel(rng, 2), synth.random_kernel(rng, 3)]
    w = synth.random_case(seed, n_ant, N, C, T, kern, fmt=fmt, extent_m=3.0, cell_m=1.0)
    w.geom.flags |= flags
    model = rng.standard_normal((C, N, N)) * 5.0
    return w, model


def _loss(w, gains, model):
    return oracle.image_loss(w.geom, w.E, gains, model)


@pytest.mark.parametrize("flags,fmt", [(0, synth.IN_C64), (synth.AUTOCORR_NONE, synth.IN_C64),
                                       (synth.NORM_PAIRS, synth.IN_C64), (0, synth.IN_CI4)])
def test_gradient_matches_finite_differences(flags, fmt):
    w, model = _case(1, flags, fmt)
    g = w.gains.astype(np.complex128)
    L0, R = _loss(w, g, model)
    grad = oracle.gain_gradient(w.geom, w.E, g, R)
    rng = np.random.default_rng(9)
    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
        Lp, _ = _loss(w, g + h * d, model)
        Lm, _ = _loss(w, g - h * d, model)
        fd = (Lp - Lm) / (2 * h)
        an = float(np.real(np.sum(np.conj(grad) * d)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_gradient_per_component():
    """Each real and imaginary part, one at a time (catches a swapped or
    conjugated component that a random direction could hide)."""
    w, model = _case(2)
    g = w.gains.astype(np.complex128)
    _, R = _loss(w, g, model)
    grad = oracle.gain_gradient(w.geom, w.E, g, R)
    h = 1e-6
    for (c, a) in [(0, 0), (1, 3), (0, 5)]:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            d = np.zeros_like(g)
            d[c, a] = unit
            fd = (_loss(w, g + h * d, model)[0] - _loss(w, g - h * d, model)[0]) / (2 * h)
            assert abs(fd - part(grad[c, a])) <= 1e-6 * max(1.0, abs(fd))


def test_gauge_orthogonality():
    """A common phase on all gains of a channel leaves its image unchanged, so
    Im sum_a conj(grad_a) g_a = 0."""
    w, model = _case(3)
    g = w.gains.astype(np.complex128)
    _, R = _loss(w, g, model)
    grad = oracle.gain_gradient(w.geom, w.E, g, R)
    for c in range(g.shape[0]):
        v = np.sum(np.conj(grad[c]) * g[c])
        assert abs(v.imag) <= 1e-10 * np.sum(np.abs(grad[c]) * np.abs(g[c]))


def test_zero_at_true_calibration():
    """Observed field = true gain x sky field, model = image of the sky field:
    the loss and its gradient vanish at g = 1 / g_true and not elsewhere."""
    w = synth.make_config(5, n_time=2, n_chan=1, grid_n=256)
    sky_geom = w.geom
    g_true = w.extra["g_true"].astype(np.complex128)
    E_sky = (w.E.astype(np.complex128) / g_true[None])
    model = oracle.moff_image(sky_geom, E_sky, None, channels=[0])
    g_opt = 1.0 / g_true
    L, R = oracle.image_loss(sky_geom, w.E, g_opt, model, channels=[0])
    grad = oracle.gain_gradient(sky_geom, w.E, g_opt, R, channels=[0])
    g_off = g_opt * (1.0 + 0.05 * np.random.default_rng(3).standard_normal(g_opt.shape))
    L1, R1 = oracle.image_loss(sky_geom, w.E, g_off, model, channels=[0])
    grad1 = oracle.gain_gradient(sky_geom, w.E, g_off, R1, channels=[0])
    assert L <= 1e-16 * L1 + 1e-12
    assert np.max(np.abs(grad)) <= 1e-6 * np.max(np.abs(grad1))
