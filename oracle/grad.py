"""FP64 gradient of an image loss with respect to the per-antenna complex gains.

TEST INFRASTRUCTURE ONLY (see `oracle.moff`).

Calibration feeds gain solutions back into the imager (Sec. 3, "Calibration":
gains are applied before gridding, and the companion EPICal method correlates
antenna signals with image pixels).  For a real loss L of the image I(g) with
pixel sensitivities R = dL/dI (a real [N, N] array per channel) this module
returns, per channel and antenna,

    grad_a = dL/dRe(g_a) + i dL/dIm(g_a) = 2 dL/d(conj g_a)

(the convention of torch's complex autograd).  With e = g E, Y_t = sum_a e_a Ghat_a
(Ghat_a the transform of antenna a's placed illumination table, as in the MOFF
image of `oracle.moff`), and the image I = s ( (1/T) sum_t |Y_t|^2
- (1/T) sum_p A_p P_p ), s the optional pair normalisation:

    dL/d(conj e_ta) = (s / T) [ sum_pix R Y_t conj(Ghat_a) - e_ta sum_pix R P_p(a) ]
    dL/d(conj g_a)  = sum_t conj(E_ta) dL/d(conj e_ta)

The first sum is the adjoint of the path: Z_t = A^H (R * Y_t) conj(A) on the
aperture cells, then sum over antenna a's footprint of conj(K) Z_t.  This is a
second implementation of the same formula as the GPU adjoint; it is pinned
independently by finite differences of the oracle's forward image
(tests/test_oracle_grad.py).
"""
from __future__ import annotations

import numpy as np

from .moff import AUTOCORR_NONE, NORM_PAIRS, calibrated_field, dft_matrix, grid_field, plan, power_pattern


def image_loss(geom, E, gains, model, channels=None):
    """L(g) = sum_{c, pix} (I_c(g) - M_c)^2 and R = dL/dI = 2 (I - M)."""
    from .moff import moff_channel
    P = plan(geom)
    if channels is None:
        channels = range(geom.freq_hz.shape[0])
    L = 0.0
    R = []
    for i, c in enumerate(channels):
        img = moff_channel(geom, E, gains, c, P)
        d = img - model[i]
        L += float(np.sum(d * d))
        R.append(2.0 * d)
    return L, np.stack(R)


def gain_gradient(geom, E, gains, R, channels=None):
    """complex128 [len(channels), n_ant]: dL/dRe(g) + i dL/dIm(g) for pixel
    sensitivities R (float [len(channels), N, N])."""
    P = plan(geom)
    N, L = P["N"], P["L"]
    flags = int(geom.flags)
    if channels is None:
        channels = range(geom.freq_hz.shape[0])
    A = dft_matrix(N, L)                                    # [N, L]
    Pp = np.stack([power_pattern(K, N) for K in P["kernels"]])
    out = []
    n_ant = geom.ant_xy.shape[0]
    for i, c in enumerate(channels):
        e = calibrated_field(E, gains, flags, c)               # [T, Na]
        Eraw = calibrated_field(E, None, flags, c)
        T = e.shape[0]
        Rc = np.asarray(R[i], dtype=np.float64)
        Eg = grid_field(e, P)                                  # [T, L, L]
        Y = np.matmul(np.matmul(A, Eg), A.T)                   # [T, N, N]
        Zt = np.matmul(np.matmul(A.conj().T, Rc[None] * Y), A.conj())   # [T, L, L] adjoint of the transform
        d = np.zeros((T, n_ant), complex)
        for a in range(n_ant):
            K = P["kernels"][P["ant_ktype"][a]]
            k = K.shape[0]
            y0, x0 = P["iy0"][a], P["ix0"][a]
            d[:, a] = np.sum(np.conj(K)[None] * Zt[:, y0:y0 + k, x0:x0 + k], axis=(1, 2))
        if not (flags & AUTOCORR_NONE):
            rho = np.array([np.sum(Rc * Pp[p]) for p in range(P["n_types"])])
            d = d - e * rho[P["ant_ktype"]][None, :]
        s = 1.0
        if flags & NORM_PAIRS:
            s = 1.0 / (n_ant * (n_ant - 1))
        out.append(2.0 * (s / T) * np.sum(np.conj(Eraw) * d, axis=0))
    return np.stack(out)
