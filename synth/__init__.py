"""Seeded synthetic workloads for the MOFF imager.

This module only *draws* inputs: antenna layouts, illumination tables, channel
frequencies, complex gains and antenna E-field streams.  It holds none of the
imaging arithmetic (no gridding, no Fourier transform, no squaring, no
accumulation); both the FP64 oracle and the HIP library consume what it returns.

The E-field of an antenna is a sum of plane waves from point sources
(Section 2, propagated-field and measured-field equations, with isotropic
antenna response) plus circular-Gaussian receiver/diffuse noise:

    E[t, c, a] = sum_s sqrt(F_s) exp(i phi[s,t,c]) exp(-2 pi i (x_a l_s + y_a m_s) / lambda_c)
                 + n[t, c, a]

with random phases phi drawn uniformly per (source, time, channel), which makes
the sources spatially coherent but temporally stochastic, as in Section 4.1.
The paper's MWA layout and LWA1 recordings are not available, so every workload
is synthetic and stands in for them with their shapes (Table 1, Section 4.4).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C_LIGHT = 299792458.0

# Flag bits shared with the C ABI (input format, autocorrelation handling and
# normalisation).  Duplicated here only as plain integers describing the input
# encoding; no arithmetic of the method depends on them in this module.
IN_C64 = 0
IN_CI4 = 1
AUTOCORR_NONE = 2
NORM_PAIRS = 4
MFMA_F16 = 8
MFMA_BF16 = 16
AUTOCORR_UV = 32


@dataclasses.dataclass
class Geometry:
    """Problem statement of the imager (Section 3, antenna-to-grid mapping).

    ant_xy    : float64 [Na, 2]  antenna positions in metres (x -> l, y -> m)
    ktype_k   : list of kernel sides k_p (square k x k tables)
    ktype_vals: list of complex64 [k_p, k_p] aperture illumination tables,
                row index u along y, column index v along x
    ant_ktype : int32 [Na] kernel type of each antenna
    freq_hz   : float64 [C] channel centre frequencies
    grid_n    : FFT side after two-fold zero padding (power of two)
    cell_m    : grid spacing in metres; 0 selects the default rule
    flags     : input format / autocorrelation / normalisation bits
    """

    ant_xy: np.ndarray
    ktype_k: List[int]
    ktype_vals: List[np.ndarray]
    ant_ktype: np.ndarray
    freq_hz: np.ndarray
    grid_n: int
    cell_m: float = 0.0
    flags: int = IN_C64

    @property
    def n_ant(self) -> int:
        return int(self.ant_xy.shape[0])

    @property
    def n_chan(self) -> int:
        return int(self.freq_hz.shape[0])

    @property
    def n_ktypes(self) -> int:
        return len(self.ktype_k)


@dataclasses.dataclass
class Workload:
    name: str
    geom: Geometry
    E: np.ndarray                 # complex64 [T, C, Na] or uint8 [T, C, Na] (4+4-bit)
    gains: Optional[np.ndarray]   # complex64 [C, Na] or None (unit gains)
    n_time: int
    extra: dict = dataclasses.field(default_factory=dict)


# ----------------------------------------------------------------------------
# layouts
# ----------------------------------------------------------------------------

def uniform_square(rng, n, side):
    return rng.uniform(0.0, side, size=(n, 2))


def uniform_disc(rng, n, diameter):
    r = 0.5 * diameter * np.sqrt(rng.uniform(0.0, 1.0, size=n))
    th = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def hex_packed(n, pitch):
    """The n points of a triangular (hex-packed) lattice nearest the origin.

    Ties in distance are broken by polar angle, then by generation index, so
    the selection is deterministic.
    """
    span = int(math.ceil(math.sqrt(n))) + 4
    pts = []
    for j in range(-span, span + 1):
        for i in range(-span, span + 1):
            pts.append((i + 0.5 * j, j * math.sqrt(3.0) / 2.0))
    pts = np.asarray(pts, dtype=np.float64) * pitch
    d = np.round(np.hypot(pts[:, 0], pts[:, 1]) / pitch, 9)
    ang = np.round(np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * np.pi), 9)
    order = np.lexsort((np.arange(len(pts)), ang, d))
    return pts[order[:n]].copy()


# ----------------------------------------------------------------------------
# illumination tables (input data: the aperture illumination of Section 3)
# ----------------------------------------------------------------------------

def kernel_tophat(k):
    return np.ones((k, k), dtype=np.complex64)


def kernel_dipole3():
    w = np.array([0.5, 1.0, 0.5])
    return np.outer(w, w).astype(np.complex64)


def kernel_airy_like(k=7):
    h = (k - 1) / 2.0
    u = np.arange(k) - h
    rho = np.hypot(u[:, None], u[None, :])
    return np.maximum(0.0, 1.0 - (rho / (k / 2.0)) ** 2).astype(np.complex64)


def channel_centres(f_lo, f_hi, n_chan):
    return f_lo + (np.arange(n_chan) + 0.5) * (f_hi - f_lo) / n_chan


# ----------------------------------------------------------------------------
# E-field streams
# ----------------------------------------------------------------------------

def draw_sources(rng, n_src, flux_lo, flux_hi, lm_max=0.9):
    r = lm_max * np.sqrt(rng.uniform(0.0, 1.0, size=n_src))
    th = rng.uniform(0.0, 2.0 * np.pi, size=n_src)
    lm = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    flux = rng.uniform(flux_lo, flux_hi, size=n_src)
    return lm, flux


def efield_stream(rng, ant_xy, freq_hz, n_time, src_lm, src_flux, noise_var,
                  dtype=np.complex64):
    """Point-source plane waves with random per-sample phases plus CN noise."""
    T, C, Na, S = n_time, len(freq_hz), ant_xy.shape[0], len(src_flux)
    out = np.empty((T, C, Na), dtype=dtype)
    amp = np.sqrt(src_flux)
    for c in range(C):
        lam = C_LIGHT / freq_hz[c]
        # geometric phase of each source at each antenna
        geo = np.exp(-2j * np.pi * (np.outer(src_lm[:, 0], ant_xy[:, 0])
                                    + np.outer(src_lm[:, 1], ant_xy[:, 1])) / lam)  # [S, Na]
        ph = np.exp(1j * rng.uniform(0.0, 2 * np.pi, size=(T, S)))                 # [T, S]
        sig = (ph * amp[None, :]) @ geo                                             # [T, Na]
        if noise_var > 0:
            s = math.sqrt(noise_var / 2.0)
            sig = sig + s * (rng.standard_normal((T, Na)) + 1j * rng.standard_normal((T, Na)))
        out[:, c, :] = sig
    return out


def quantise_ci4(E, rms_levels=2.0):
    """Encode complex samples as one byte: real = high nibble, imag = low nibble,
    both two's complement in [-8, 7], after scaling to the given per-component
    RMS in quantisation levels."""
    Ef = E.astype(np.complex128)
    rms = math.sqrt(float(np.mean(Ef.real ** 2 + Ef.imag ** 2)) / 2.0)
    s = rms_levels / rms if rms > 0 else 1.0
    re = np.clip(np.rint(Ef.real * s), -8, 7).astype(np.int16)
    im = np.clip(np.rint(Ef.imag * s), -8, 7).astype(np.int16)
    return (((re & 0xF) << 4) | (im & 0xF)).astype(np.uint8)


def random_gains(rng, n_chan, n_ant, amp_lo=0.8, amp_hi=1.2):
    amp = rng.uniform(amp_lo, amp_hi, size=(n_chan, n_ant))
    ph = rng.uniform(-np.pi, np.pi, size=(n_chan, n_ant))
    return (amp * np.exp(1j * ph)).astype(np.complex64)


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

CONFIG_NAMES = {
    1: "tiny: 16 ant in 8 m box, 2x2 tophat, 1 ch @ 60 MHz, T=64, N=32, c64",
    2: "LWA-shaped: 256 ant in 100 m disc, 3x3 dipole, 128 ch 40-80 MHz, T=1000, N=128, ci4",
    3: "HERA-shaped: 350 hex 14.6 m, 7x7 Airy-like, 1024 ch 100-200 MHz, T=256, N=256, ci4",
    4: "reduced-precision: LWA layout, 128 ch 40-80 MHz, T=1000, N=64/128",
    5: "calibration: 1024 ant in 400 m disc, 70% 3x3 / 30% 7x7, 256 ch 100-200 MHz, T=128, N=256, c64 + gains",
}

DEFAULT_SEED = {1: 0, 2: 2, 3: 3, 4: 4, 5: 5}
FULL_SHAPE = {  # (T, C, N)
    1: (64, 1, 32),
    2: (1000, 128, 128),
    3: (256, 1024, 256),
    4: (1000, 128, 128),
    5: (128, 256, 256),
}


def make_config(cfg: int, seed: Optional[int] = None, n_time: Optional[int] = None,
                n_chan: Optional[int] = None, grid_n: Optional[int] = None,
                in_format: Optional[int] = None) -> Workload:
    """Draw workload `cfg` (1..5).  n_time / n_chan / grid_n shrink it for tests
    (channels keep the full band: a reduced channel count samples it evenly)."""
    if seed is None:
        seed = DEFAULT_SEED[cfg]
    T_full, C_full, N_full = FULL_SHAPE[cfg]
    T = T_full if n_time is None else int(n_time)
    C = C_full if n_chan is None else int(n_chan)
    N = N_full if grid_n is None else int(grid_n)
    rng = np.random.default_rng(seed)
    gains = None
    extra = {}

    if cfg == 1:
        xy = uniform_square(rng, 16, 8.0)
        kt = [kernel_tophat(2)]
        ant_t = np.zeros(16, np.int32)
        freq = np.array([60e6]) if C == 1 else channel_centres(55e6, 65e6, C)
        src_lm, src_f = draw_sources(rng, 3, 1.0, 10.0)
        noise = 0.1
        fmt = IN_C64
    elif cfg in (2, 4):
        xy = uniform_disc(rng, 256, 100.0)
        kt = [kernel_dipole3()]
        ant_t = np.zeros(256, np.int32)
        freq = channel_centres(40e6, 80e6, C)
        src_lm, src_f = draw_sources(rng, 20, 1.0, 10.0)
        noise = 1.0
        fmt = IN_CI4 if cfg == 2 else IN_C64
    elif cfg == 3:
        xy = hex_packed(350, 14.6)
        kt = [kernel_airy_like(7)]
        ant_t = np.zeros(350, np.int32)
        freq = channel_centres(100e6, 200e6, C)
        src_lm, src_f = draw_sources(rng, 20, 1.0, 10.0)
        noise = 1.0
        fmt = IN_CI4
    elif cfg == 5:
        xy = uniform_disc(rng, 1024, 400.0)
        kt = [kernel_dipole3(), kernel_airy_like(7)]
        ant_t = np.zeros(1024, np.int32)
        ant_t[rng.permutation(1024)[:307]] = 1
        freq = channel_centres(100e6, 200e6, C)
        src_lm, src_f = draw_sources(rng, 20, 1.0, 10.0)
        noise = 0.1
        fmt = IN_C64
    else:
        raise ValueError(f"unknown config {cfg}")

    if in_format is not None:
        fmt = in_format
    geom = Geometry(ant_xy=xy.astype(np.float64), ktype_k=[int(k.shape[0]) for k in kt],
                    ktype_vals=kt, ant_ktype=ant_t, freq_hz=np.asarray(freq, np.float64),
                    grid_n=N, cell_m=0.0, flags=fmt)
    E = efield_stream(rng, xy, geom.freq_hz, T, src_lm, src_f, noise)
    if cfg == 5:
        g_true = random_gains(rng, C, 1024)
        E = (E * g_true[None, :, :]).astype(np.complex64)   # observed = true gain x sky field
        gains = (1.0 / g_true).astype(np.complex64)        # calibration that undoes them
        extra["g_true"] = g_true
    if fmt == IN_CI4:
        E = quantise_ci4(E)
    extra["src_lm"] = src_lm
    extra["src_flux"] = src_f
    return Workload(name=CONFIG_NAMES[cfg], geom=geom, E=E, gains=gains, n_time=T, extra=extra)


def random_case(seed: int, n_ant: int, grid_n: int, n_chan: int, n_time: int,
                kernels: List[np.ndarray], fmt: int = IN_C64, with_gains: bool = True,
                extent_m: float = 8.0, freq_lo: float = 50e6, freq_hi: float = 80e6,
                cell_m: float = 0.0) -> Workload:
    """A small random problem with arbitrary (possibly complex, asymmetric)
    illumination tables, used for edge cases and ragged shapes."""
    rng = np.random.default_rng(seed)
    xy = uniform_square(rng, n_ant, extent_m)
    ant_t = rng.integers(0, len(kernels), size=n_ant).astype(np.int32)
    freq = channel_centres(freq_lo, freq_hi, n_chan)
    geom = Geometry(ant_xy=xy, ktype_k=[int(k.shape[0]) for k in kernels],
                    ktype_vals=[np.asarray(k, np.complex64) for k in kernels],
                    ant_ktype=ant_t, freq_hz=freq, grid_n=grid_n, cell_m=cell_m, flags=fmt)
    E = (rng.standard_normal((n_time, n_chan, n_ant))
         + 1j * rng.standard_normal((n_time, n_chan, n_ant))).astype(np.complex64)
    if fmt == IN_CI4:
        E = quantise_ci4(E)
    gains = random_gains(rng, n_chan, n_ant) if with_gains else None
    return Workload(name=f"random seed={seed}", geom=geom, E=E, gains=gains, n_time=n_time)


def random_kernel(rng, k, complex_valued=True):
    re = rng.uniform(-1.0, 1.0, size=(k, k))
    im = rng.uniform(-1.0, 1.0, size=(k, k)) if complex_valued else 0.0
    return (re + 1j * im).astype(np.complex64)
