"""FP64 oracle of the paper's uv-plane autocorrelation removal (Sec. 4.2).

TEST INFRASTRUCTURE ONLY (see `oracle.moff`).

Squaring the gridded field leaves every antenna's correlation with itself in the
image; in the uv plane these autocorrelations sit around the zero-spacing
pixel, with the shape of each antenna's illumination table correlated with
itself.  The paper removes them once per integration, in this order:

  1. take the time-averaged squared image P = S / T back to the uv plane with
     the inverse of the image transform;
  2. estimate the autocorrelation kernel from the aperture illumination tables
     (the gridding step already has them);
  3. subtract that kernel, centred on the zero-spacing pixel and scaled to the
     data's value there;
  4. transform the result back to the image plane.

Readings (the paper is terse here): the uv data are
    D[d] = (1/N^2) sum_pix P[pix] exp(-2 pi i d . (pix - N/2) / N),
which inverts the unnormalised image transform, so D is the sum over all
antenna pairs of the gridded-field correlations at lag d (lags taken modulo N;
they span -(N/2 - 1) .. N/2 - 1, so nothing aliases).  The kernel estimate for a
heterogeneous array sums each antenna's table autocorrelation,
    a[d] = sum_p n_p sum_u K_p[u + d] conj(K_p[u])   (n_p antennas of type p),
which is the paper's single-table kernel times n when all antennas share one
table.  "Scaled to the peak value" is read as alpha = D[0] / a[0], so the
corrected uv data are zero at zero spacing.  The pair normalisation flag
applies to the result as for the exact removal.

The steps are taken literally, with explicit DFT matrices and an explicit
table autocorrelation; no closed form is used.
"""
from __future__ import annotations

import numpy as np

from .moff import NORM_PAIRS, calibrated_field, grid_field, image_field, plan


def _lag_dft(N):
    """B[pix, d] = exp(+2 pi i d (pix - N/2) / N) for pix, d in [0, N)."""
    pix = np.arange(N)[:, None] - N // 2
    d = np.arange(N)[None, :]
    return np.exp(2j * np.pi * ((pix * d) % N) / N)


def table_autocorrelation(K, N):
    """a[d] = sum_u K[u + d] conj(K[u]) on an N x N lag grid (lags modulo N)."""
    k = K.shape[0]
    a = np.zeros((N, N), complex)
    for dy in range(-(k - 1), k):
        for dx in range(-(k - 1), k):
            s = 0.0 + 0.0j
            for uy in range(k):
                for ux in range(k):
                    vy, vx = uy + dy, ux + dx
                    if 0 <= vy < k and 0 <= vx < k:
                        s += K[vy, vx] * np.conj(K[uy, ux])
            a[dy % N, dx % N] += s
    return a


def uv_channel(geom, E, gains, channel, P=None, keep=False):
    """Time-averaged image of one channel with the autocorrelations removed by
    the uv-plane rule, float64 [N, N]."""
    if P is None:
        P = plan(geom)
    N = P["N"]
    flags = int(geom.flags)
    e = calibrated_field(E, gains, flags, channel)          # [T, Na]
    T = e.shape[0]
    Y = image_field(grid_field(e, P), N)                     # [T, N, N]
    Pbar = np.sum((Y * Y.conj()).real, axis=0) / T           # S / T, autocorrelations included

    B = _lag_dft(N)                                          # image <- uv
    Binv = np.conj(B) / N                                    # uv <- image (per axis)
    D = Binv.T @ Pbar @ Binv                                 # step 1: D[dy, dx]

    counts = np.bincount(P["ant_ktype"], minlength=P["n_types"])
    a = sum(counts[p] * table_autocorrelation(P["kernels"][p], N) for p in range(P["n_types"]))   # step 2
    alpha = D[0, 0].real / a[0, 0].real                      # step 3: scaled to the zero-spacing value
    D2 = D - alpha * a

    img = (B @ D2 @ B.T).real                                # step 4
    if flags & NORM_PAIRS:
        na = e.shape[1]
        img = img / (na * (na - 1))
    if keep:
        return img, dict(D=D, a=a, alpha=alpha, Pbar=Pbar)
    return img


def uv_image(geom, E, gains=None, channels=None):
    P = plan(geom)
    if channels is None:
        channels = range(geom.freq_hz.shape[0])
    return np.stack([uv_channel(geom, E, gains, c, P) for c in channels])
