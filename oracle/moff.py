"""FP64 CPU oracle for the MOFF direct-imaging hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product library never
does, and there is no CPU fallback in the product path.  It shares no code with
the HIP library: it reads the same seeded inputs and recomputes everything from
the paper's definitions, in float64 / complex128, slowly and plainly.

What it computes, per frequency channel c (Sec. 2, MOFF imaging equation,
eq. dirty-image-MOFF; Sec. 3 implementation steps; Sec. 4.2 autocorrelations):

  1. antenna-to-grid mapping (Sec. 3, "Antenna-to-Grid Mapping"):
     a regular grid of spacing cell_m in the antenna coordinate frame, each
     antenna's k x k illumination table placed at the nearest grid cells;
  2. calibration (Sec. 3, "Calibration"): e = g * E, applied before gridding;
  3. gridding (Sec. 3, "Gridding Convolution", E(r) = M(r,a) E(a)):
     Eg[iy0_a+u, ix0_a+v] += K_a[u, v] * e_a over the L x L aperture quadrant;
  4. zero padding to N = 2L per axis and the spatial 2-D Fourier transform
     (Sec. 3, "Spatial Fourier Transform"), positive exponent, unnormalised:
       Y[r, q] = sum_{iy,ix} Eg[iy, ix] exp(+2 pi i (iy (r - N/2) + ix (q - N/2)) / N)
     so pixel (N/2, N/2) is l = m = 0, rows follow m (y), columns follow l (x);
  5. squaring and time averaging (Sec. 3, "Time-averaging"): S = sum_t |Y|^2;
  6. removal of each antenna's own power (Sec. 4.2: the per-antenna subtraction
     named as the general solution): A_p = sum_t sum_{a of type p} |e_a|^2 and
     P_p = |sum_{u,v} K_p[u,v] exp(+2 pi i (u (r-N/2) + v (q-N/2)) / N)|^2,
       I = (S - sum_p A_p P_p) / T,
     optionally times 1 / (Na (Na - 1)) (Sec. 5, eq. wt-dirty-image-EPIC).

Readings taken where the paper is silent are listed in the repository design
notes; the ones that change numbers are: the default cell size rule
(`default_cell_size`), round-half-up nearest-cell placement, the 4+4-bit input
encoding, and exact per-antenna self-power subtraction.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np

C_LIGHT = 299792458.0

IN_C64 = 0
IN_CI4 = 1
AUTOCORR_NONE = 2
NORM_PAIRS = 4


class FootprintOverflow(ValueError):
    """Antenna footprints do not fit in the N/2 x N/2 aperture region."""


# ----------------------------------------------------------------------------
# step 1: the grid and the antenna-to-grid mapping
# ----------------------------------------------------------------------------

def default_cell_size(ant_xy, k_ant, freq_hz, grid_n):
    """Grid spacing when the caller gives none (Sec. 3, antenna-to-grid mapping,
    and Sec. 6.1, field-of-view grid).

    The paper's default is at most half the shortest wavelength.  When the
    array does not fit in the aperture region at that spacing, the spacing is
    widened just enough that the span of the layout plus the widest footprint
    (and one cell of rounding slack) fits in N/2 cells.
    """
    lam_min = C_LIGHT / float(np.max(freq_hz))
    span = max(float(np.ptp(ant_xy[:, 0])), float(np.ptp(ant_xy[:, 1])))
    room = grid_n // 2 - int(np.max(k_ant)) - 1
    if room <= 0:
        raise FootprintOverflow("grid too small for the largest footprint")
    return max(lam_min / 2.0, span / room)


def cell_indices(ant_xy, k_ant, cell_m, grid_n):
    """Lower-left grid cell of each antenna footprint (Sec. 3: nearest-neighbour
    mapping of the footprint onto the regular grid).

    A k x k footprint centred on x/cell_m covers cells ix0 .. ix0+k-1 whose
    centre (ix0 + (k-1)/2) is the one nearest the antenna, ties rounding up:
        ix0 = floor(x / cell_m - (k - 1) / 2 + 0.5)
    Indices are then shifted so the smallest is 0 on each axis.
    """
    k = np.asarray(k_ant, dtype=np.float64)
    h = (k - 1.0) / 2.0
    ix = np.floor(ant_xy[:, 0] / cell_m - h + 0.5).astype(np.int64)
    iy = np.floor(ant_xy[:, 1] / cell_m - h + 0.5).astype(np.int64)
    ix -= ix.min()
    iy -= iy.min()
    L = grid_n // 2
    kk = np.asarray(k_ant, dtype=np.int64)
    if int((ix + kk).max()) > L or int((iy + kk).max()) > L:
        raise FootprintOverflow("footprints extend beyond the aperture region")
    return ix, iy


def plan(geom):
    """Everything the path needs that does not depend on the data."""
    k_ant = np.asarray([geom.ktype_k[p] for p in geom.ant_ktype], dtype=np.int64)
    N = int(geom.grid_n)
    if N < 8 or (N & (N - 1)) != 0:
        raise ValueError("grid_n must be a power of two >= 8")
    cell = float(geom.cell_m) if geom.cell_m > 0 else default_cell_size(geom.ant_xy, k_ant, geom.freq_hz, N)
    ix0, iy0 = cell_indices(geom.ant_xy, k_ant, cell, N)
    kernels = [np.asarray(K, dtype=np.complex128) for K in geom.ktype_vals]
    return dict(N=N, L=N // 2, cell_m=cell, ix0=ix0, iy0=iy0, k_ant=k_ant,
                kernels=kernels, ant_ktype=np.asarray(geom.ant_ktype, np.int64),
                n_types=len(kernels),
                lm_per_pixel=(C_LIGHT / np.asarray(geom.freq_hz, np.float64)) / (N * cell))


# ----------------------------------------------------------------------------
# step 2: ingest and calibration
# ----------------------------------------------------------------------------

def decode_ci4(raw):
    """One byte per complex sample: real part in the high nibble, imaginary part
    in the low nibble, each a two's-complement integer in [-8, 7]."""
    b = np.asarray(raw, dtype=np.int64)
    hi = b >> 4
    lo = b & 0xF
    re = np.where(hi >= 8, hi - 16, hi)
    im = np.where(lo >= 8, lo - 16, lo)
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def calibrated_field(E, gains, flags, channel):
    """e[t, a] = g[c, a] * E[t, c, a] for one channel (Sec. 3, Calibration:
    gains are applied before gridding)."""
    if flags & IN_CI4:
        Ec = decode_ci4(E[:, channel, :])
    else:
        Ec = np.asarray(E[:, channel, :], dtype=np.complex128)
    if gains is None:
        return Ec
    return Ec * np.asarray(gains[channel], dtype=np.complex128)[None, :]


# ----------------------------------------------------------------------------
# step 3: gridding
# ----------------------------------------------------------------------------

def grid_field(e, P):
    """Eg[t] = M e[t]: every antenna adds its illumination table times its
    calibrated field at its footprint cells (Sec. 3, gridding convolution)."""
    T = e.shape[0]
    L = P["L"]
    Eg = np.zeros((T, L, L), dtype=np.complex128)
    for a in range(e.shape[1]):
        K = P["kernels"][P["ant_ktype"][a]]
        k = K.shape[0]
        y0, x0 = P["iy0"][a], P["ix0"][a]
        Eg[:, y0:y0 + k, x0:x0 + k] += K[None, :, :] * e[:, a][:, None, None]
    return Eg


# ----------------------------------------------------------------------------
# step 4: zero padding + 2-D Fourier transform, by direct DFT
# ----------------------------------------------------------------------------

def dft_matrix(N, n_in):
    """A[r, n] = exp(+2 pi i n (r - N/2) / N) for output r < N, input n < n_in.
    The integer phase n (r - N/2) is reduced mod N before the float64 angle."""
    r = np.arange(N, dtype=np.int64)[:, None] - N // 2
    n = np.arange(n_in, dtype=np.int64)[None, :]
    ph = np.mod(n * r, N).astype(np.float64)
    return np.exp(2j * np.pi * ph / N)


def image_field(Eg, N):
    """Y = A Eg A^T: the direct DFT of the zero-padded grid, one matrix product
    per axis (the same double sum as `image_field_literal`)."""
    A = dft_matrix(N, Eg.shape[-1])
    return np.matmul(np.matmul(A, Eg), A.T)


def image_field_literal(Eg, N):
    """The per-pixel double sum, written out (tiny grids only)."""
    L = Eg.shape[-1]
    Y = np.zeros(Eg.shape[:-2] + (N, N), dtype=np.complex128)
    iy = np.arange(L)[:, None]
    ix = np.arange(L)[None, :]
    for r in range(N):
        for q in range(N):
            w = np.exp(2j * np.pi * (iy * (r - N // 2) + ix * (q - N // 2)) / N)
            Y[..., r, q] = np.sum(Eg * w, axis=(-2, -1))
    return Y


# ----------------------------------------------------------------------------
# step 6 ingredients: per-antenna self power
# ----------------------------------------------------------------------------

def power_pattern(K, N):
    """P[r, q] = |DFT_N of the k x k table|^2 with the same sign and origin as
    the image (Sec. 4.2: the antenna power response in the image plane)."""
    A = dft_matrix(N, K.shape[0])
    B = A @ np.asarray(K, np.complex128) @ A.T
    return (B * B.conj()).real


def self_power(e, ant_ktype, n_types):
    """A_p = sum_t sum_{a of type p} |e_a(t)|^2."""
    pw = np.sum((e * e.conj()).real, axis=0)
    return np.array([pw[ant_ktype == p].sum() for p in range(n_types)], dtype=np.float64)


# ----------------------------------------------------------------------------
# the whole path
# ----------------------------------------------------------------------------

def moff_channel(geom, E, gains, channel, P=None, keep=False):
    """Time-averaged MOFF image of one channel, float64 [N, N]."""
    if P is None:
        P = plan(geom)
    N = P["N"]
    flags = int(geom.flags)
    e = calibrated_field(E, gains, flags, channel)              # [T, Na]
    T = e.shape[0]
    Eg = grid_field(e, P)                                      # [T, L, L]
    Y = image_field(Eg, N)                                     # [T, N, N]
    S = np.sum((Y * Y.conj()).real, axis=0)                    # sum_t |Y|^2
    A = self_power(e, P["ant_ktype"], P["n_types"])
    Pp = np.stack([power_pattern(K, N) for K in P["kernels"]])
    if flags & AUTOCORR_NONE:
        img = S / T
    else:
        img = (S - np.tensordot(A, Pp, axes=1)) / T
    if flags & NORM_PAIRS:
        na = e.shape[1]
        img = img / (na * (na - 1))
    if keep:
        return img, dict(e=e, Eg=Eg, Y=Y, S=S, A=A, P=Pp)
    return img


def moff_image(geom, E, gains=None, channels: Optional[Sequence[int]] = None):
    """Image cube float64 [len(channels), N, N] (all channels by default)."""
    P = plan(geom)
    if channels is None:
        channels = range(geom.freq_hz.shape[0])
    return np.stack([moff_channel(geom, E, gains, c, P) for c in channels])
