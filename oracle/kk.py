"""Kramers-Kronig field recovery from one NA-matched image (Sec. 2.3, Eq. 4-7).

Eq. 4 forms the logarithm of the shifted field times exp(-j theta_i); its real
part is half the log intensity.  Eq. 5 keeps the transform of log I on the open
half plane k.k_i < 0, halves it on the line k.k_i = 0 and drops it elsewhere
(the directional Hilbert transform).  Eq. 6 exponentiates the inverse
transform; Eq. 7 transforms the recovered field, whose support is
Circ(k + k_i).

Readings taken (the paper is silent or garbled here):
* Eq. 4's imaginary part is arg S'_i - theta_i and Eq. 3's ramp carries j;
* the sign of k.k_i is the exact integer dot product in signed FFT indices
  (the -N/2 bins stay negative);
* log of a non-positive value: the intensity is floored at
  eps = log_floor_rel * mean(I) before the log;
* the recovered spectrum is multiplied by Circ(k + k_i) (Eq. 7's support)
  before any later step uses it.
"""

import numpy as np

from .grid import k_grid, circ


def half_plane_mask(n, k_i):
    """Eq. 5's weights: 1 where k.k_i < 0, 1/2 where k.k_i = 0, 0 where > 0."""
    ky, kx = k_grid(n)
    dot = kx * int(k_i[0]) + ky * int(k_i[1])
    return np.where(dot < 0, 1.0, np.where(dot == 0, 0.5, 0.0))


def kk_field(intensity, k_i, log_floor_rel=1e-6):
    """Recovered spatial field S'_i(x) exp(-j theta_i) (Eq. 4-6), no support mask.

    Returns (field, floor_hit) where floor_hit says whether any pixel was
    clamped to the log floor.
    """
    img = np.asarray(intensity, dtype=np.float64)
    n = img.shape[0]
    eps = log_floor_rel * img.mean()
    floor_hit = bool(np.any(img < eps))
    log_i = np.log(np.maximum(img, eps))
    g = np.fft.fft2(log_i) * half_plane_mask(n, k_i)
    return np.exp(np.fft.ifft2(g)), floor_hit


def kk_spectrum(intensity, k_i, r, log_floor_rel=1e-6):
    """KK spectrum s_hat_i(k) = fft2(field) Circ(k + k_i) (Eq. 7)."""
    field, _ = kk_field(intensity, k_i, log_floor_rel)
    n = field.shape[0]
    ky, kx = k_grid(n)
    support = circ(ky + int(k_i[1]), kx + int(k_i[0]), r)
    return np.fft.fft2(field) * support
