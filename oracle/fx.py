"""FP64 visibility-based (FX) imaging routes, used to pin the MOFF oracle.

TEST INFRASTRUCTURE ONLY (see `oracle.moff`).

Sec. 2 shows that the MOFF image (eq. dirty-image-MOFF) equals the software-
holography image made from visibilities (eq. dirty-image-FX, with the e-field
convolution identity eq. e-field-conv): cross-multiply antenna pairs
(eq. cc-vis), grid each visibility with the pair's power response
B_ab = cross-correlation of the two aperture illuminations, and Fourier
transform once per integration.  Two versions:

* `fx_discrete_image` grids each visibility with the cross-correlation of the
  two *placed, discrete* footprints.  Without the zero-spacing (a == b) terms it
  must equal the MOFF image with self power removed, to rounding.
* `fx_analytic_image` samples the continuous cross-correlation of two square
  top-hat apertures at the true baseline instead (Sec. 4.3: the visibility
  route samples B_ab directly, centred on the baseline).  It differs from MOFF
  only by gridding coarseness and converges to it as the grid is refined.
"""
from __future__ import annotations

import numpy as np

from .moff import AUTOCORR_NONE, NORM_PAIRS, calibrated_field, plan


def visibilities(e):
    """V_ab = <e_a conj(e_b)>_t over the integration (eq. cc-vis)."""
    T = e.shape[0]
    return (e.T @ e.conj()) / T


def kernel_xcorr(Ka, Kb):
    """X[du + kb - 1, dv + kb - 1] = sum_{u,v} Ka[u, v] conj(Kb[u - du, v - dv]):
    the lag response of a pair whose footprints start at the same cell."""
    ka, kb = Ka.shape[0], Kb.shape[0]
    X = np.zeros((ka + kb - 1, ka + kb - 1), dtype=np.complex128)
    for u in range(ka):
        for v in range(ka):
            for u2 in range(kb):
                for v2 in range(kb):
                    X[u - u2 + kb - 1, v - v2 + kb - 1] += Ka[u, v] * np.conj(Kb[u2, v2])
    return X


def lag_dft_matrix(N, L):
    """D[r, j] = exp(+2 pi i d (r - N/2) / N) for lags d = j - (L - 1), |d| < L."""
    r = np.arange(N, dtype=np.int64)[:, None] - N // 2
    d = np.arange(2 * L - 1, dtype=np.int64)[None, :] - (L - 1)
    ph = np.mod(d * r, N).astype(np.float64)
    return np.exp(2j * np.pi * ph / N)


def _finish(R, P, flags, n_ant):
    N, L = P["N"], P["L"]
    D = lag_dft_matrix(N, L)
    img = (D @ R @ D.T).real
    if flags & NORM_PAIRS:
        img = img / (n_ant * (n_ant - 1))
    return img


def fx_discrete_image(geom, E, gains, channel, include_autos=None):
    """Visibility-route image on the lag grid of the discrete footprints."""
    P = plan(geom)
    flags = int(geom.flags)
    if include_autos is None:
        include_autos = bool(flags & AUTOCORR_NONE)
    e = calibrated_field(E, gains, flags, channel)
    V = visibilities(e)
    L = P["L"]
    na = e.shape[1]
    R = np.zeros((2 * L - 1, 2 * L - 1), dtype=np.complex128)
    types = P["ant_ktype"]
    kern = P["kernels"]
    for p in range(P["n_types"]):
        for q in range(P["n_types"]):
            X = kernel_xcorr(kern[p], kern[q])
            kb = kern[q].shape[0]
            A = np.nonzero(types == p)[0]
            B = np.nonzero(types == q)[0]
            if A.size == 0 or B.size == 0:
                continue
            aa, bb = np.meshgrid(A, B, indexing="ij")
            aa = aa.ravel()
            bb = bb.ravel()
            if not include_autos:
                keep = aa != bb
                aa, bb = aa[keep], bb[keep]
            v = V[aa, bb]
            oy = P["iy0"][aa] - P["iy0"][bb] - (kb - 1) + (L - 1)
            ox = P["ix0"][aa] - P["ix0"][bb] - (kb - 1) + (L - 1)
            for du in range(X.shape[0]):
                for dv in range(X.shape[1]):
                    if X[du, dv] == 0:
                        continue
                    np.add.at(R, (oy + du, ox + dv), v * X[du, dv])
    return _finish(R, P, flags, na)


def tophat_xcorr_area(dx, dy, side):
    """Continuous cross-correlation of two side x side squares at offset (dx, dy)."""
    return np.clip(side - np.abs(dx), 0, None) * np.clip(side - np.abs(dy), 0, None)


def fx_analytic_image(geom, E, gains, channel, side_m):
    """Visibility route with B_ab sampled analytically at the true baseline, for
    identical square top-hat apertures of side `side_m` metres.  The sampled
    response is divided by the cell area so that it has the same scale as the
    discrete footprint cross-correlation (k^2 at zero lag for a k-cell square)."""
    P = plan(geom)
    flags = int(geom.flags)
    e = calibrated_field(E, gains, flags, channel)
    V = visibilities(e)
    L = P["L"]
    cell = P["cell_m"]
    na = e.shape[1]
    xy = np.asarray(geom.ant_xy, np.float64)
    # the MOFF grid origin: the cell that antenna 0's footprint centre maps to
    # is fixed by the global shift, which only rotates the image phase and
    # cancels in the pair products; baselines are all that matter here.
    R = np.zeros((2 * L - 1, 2 * L - 1), dtype=np.complex128)
    d = (np.arange(2 * L - 1) - (L - 1)) * cell
    for a in range(na):
        for b in range(na):
            if a == b:
                continue
            bx = xy[a, 0] - xy[b, 0]
            by = xy[a, 1] - xy[b, 1]
            wy = np.clip(side_m - np.abs(d - by), 0, None)
            wx = np.clip(side_m - np.abs(d - bx), 0, None)
            R += V[a, b] * np.outer(wy, wx) / (cell * cell)
    return _finish(R, P, flags, na)
