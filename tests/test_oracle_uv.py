"""Pins of the oracle's uv-plane autocorrelation removal (Sec. 4.2) against
facts the paper and the mathematics fix, independent of its own steps:

* the uv data at lag d are the gridded field's correlation with itself at lag
  d, summed over all antenna pairs and averaged in time (brute force);
* for one illumination table and footprints that never overlap, the uv rule
  removes exactly each antenna's own power, so it equals the per-antenna
  subtraction (Sec. 4.2 calls that the general solution);
* after the subtraction the zero-spacing pixel is empty, so the image sums to
  zero;
* whatever the layout, the uv rule differs from the per-antenna subtraction only
  by a combination of the antenna power patterns P_p (both subtract multiples
  of the tables' autocorrelations).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import uv_autocorr


def _lattice_case(seed, k, spacing, n_side, N, T=4, C=1):
    """Homogeneous array on a square lattice `spacing` cells apart (cell 1 m)."""
    rng = np.random.default_rng(seed)
    g = np.arange(n_side, dtype=np.float64) * spacing
    xy = np.stack(np.meshgrid(g, g), -1).reshape(-1, 2) + 0.25
    K = synth.random_kernel(rng, k)
    geom = synth.Geometry(ant_xy=xy, ktype_k=[k], ktype_vals=[K], ant_ktype=np.zeros(len(xy), np.int32),
                          freq_hz=np.array([60e6] * C), grid_n=N, cell_m=1.0, flags=synth.IN_C64)
    E = (rng.standard_normal((T, C, len(xy))) + 1j * rng.standard_normal((T, C, len(xy)))).astype(np.complex64)
    gains = synth.random_gains(rng, C, len(xy))
    return synth.Workload(name="lattice", geom=geom, E=E, gains=gains, n_time=T)


def _hetero_case(seed=3, N=32, extent=9.0, n_ant=14):
    rng = np.random.default_rng(seed)
    return synth.random_case(seed, n_ant, N, 1, 5, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 2)],
                             extent_m=extent, cell_m=1.0)


def test_uv_data_are_the_field_autocorrelation():
    w = _hetero_case(N=16, extent=4.0, n_ant=6)
    P = oracle.plan(w.geom)
    N, L = P["N"], P["L"]
    img, parts = uv_autocorr.uv_channel(w.geom, w.E, w.gains, 0, P, keep=True)
    e = oracle.calibrated_field(w.E, w.gains, w.geom.flags, 0)
    Eg = oracle.grid_field(e, P)                                  # [T, L, L]
    T = Eg.shape[0]
    ref = np.zeros((N, N), complex)
    for dy in range(-(L - 1), L):
        for dx in range(-(L - 1), L):
            s = 0.0
            for y in range(max(0, -dy), min(L, L - dy)):
                for x in range(max(0, -dx), min(L, L - dx)):
                    s = s + np.sum(Eg[:, y + dy, x + dx] * np.conj(Eg[:, y, x]))
            ref[dy % N, dx % N] = s / T
    assert np.abs(parts["D"] - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("k,spacing", [(2, 3), (3, 4), (1, 2)])
def test_equals_exact_removal_without_overlap(k, spacing):
    w = _lattice_case(7 + k, k, spacing, 4, 32)
    P = oracle.plan(w.geom)
    exact, parts = oracle.moff_channel(w.geom, w.E, w.gains, 0, P, keep=True)
    uv = uv_autocorr.uv_channel(w.geom, w.E, w.gains, 0, P)
    pbar = parts["S"] / w.E.shape[0]
    assert np.abs(uv - exact).max() <= 1e-10 * np.abs(pbar).max()


def test_heterogeneous_equal_power_weights_tables_by_count():
    """Two table types on a lattice with no overlaps and every antenna at the
    same power (unit-modulus fields and gains): the kernel estimate weights each
    type's autocorrelation by its antenna count, so the uv rule is again exact."""
    rng = np.random.default_rng(21)
    g = np.arange(5, dtype=np.float64) * 4.0
    xy = np.stack(np.meshgrid(g, g), -1).reshape(-1, 2) + 0.25
    na = len(xy)
    types = (rng.random(na) < 0.3).astype(np.int32)           # about 30 % of type 1
    K0, K1 = synth.random_kernel(rng, 2), synth.random_kernel(rng, 3)
    geom = synth.Geometry(ant_xy=xy, ktype_k=[2, 3], ktype_vals=[K0, K1], ant_ktype=types,
                          freq_hz=np.array([60e6]), grid_n=64, cell_m=1.0, flags=synth.IN_C64)
    T = 3
    E = np.exp(2j * np.pi * rng.random((T, 1, na))).astype(np.complex64)
    gains = np.exp(2j * np.pi * rng.random((1, na))).astype(np.complex64)
    P = oracle.plan(geom)
    exact, parts = oracle.moff_channel(geom, E, gains, 0, P, keep=True)
    uv = uv_autocorr.uv_channel(geom, E, gains, 0, P)
    assert np.abs(uv - exact).max() <= 1e-9 * np.abs(parts["S"] / T).max()


@pytest.mark.parametrize("case", ["hetero", "config1", "lattice_overlap"])
def test_zero_spacing_removed_and_difference_in_power_patterns(case):
    if case == "hetero":
        w = _hetero_case()
    elif case == "config1":
        w = synth.make_config(1, n_time=8)
    else:
        w = _lattice_case(5, 3, 2, 5, 32)                      # 3x3 tables 2 cells apart overlap
    P = oracle.plan(w.geom)
    uv, parts = uv_autocorr.uv_channel(w.geom, w.E, w.gains, 0, P, keep=True)
    exact = oracle.moff_channel(w.geom, w.E, w.gains, 0, P)
    scale = np.abs(parts["Pbar"]).max()
    assert abs(uv.sum()) <= 1e-10 * scale * uv.size
    N = P["N"]
    basis = np.stack([oracle.power_pattern(K, N).ravel() for K in P["kernels"]], 1)
    diff = (uv - exact).ravel()
    coef, *_ = np.linalg.lstsq(basis, diff, rcond=None)
    assert np.abs(basis @ coef - diff).max() <= 1e-9 * scale
    if case == "lattice_overlap":
        # overlapping footprints put cross-correlations on the zero-spacing
        # pixel, so the rule over-subtracts: the two removals differ
        assert np.abs(diff).max() > 1e-6 * scale


def test_pair_normalisation_applies():
    w = _hetero_case()
    P = oracle.plan(w.geom)
    a = uv_autocorr.uv_channel(w.geom, w.E, w.gains, 0, P)
    w.geom.flags |= synth.NORM_PAIRS
    b = uv_autocorr.uv_channel(w.geom, w.E, w.gains, 0, P)
    na = w.geom.ant_xy.shape[0]
    assert np.allclose(b * na * (na - 1), a, rtol=1e-12, atol=1e-12 * np.abs(a).max())
