"""Discrete frequency-grid conventions of the oracle.

The paper writes its spectra on continuous transverse k (Sec. 2.2, Eq. 1) and
refers to positions of k on a flattened grid (Sec. 2.3, text after Eq. 10)
without fixing a discretisation.  Reading taken here:

* arrays are N x N, indexed [y][x], x fastest;
* the DFT is NumPy's: ``fft2`` unnormalised with exp(-2 pi j k.n / N),
  ``ifft2`` carries 1/N^2;
* a frequency index is the signed integer pair (ky, kx) in [-N/2, N/2)^2 and
  arrays are stored in FFT order (DC at [0][0]);
* the pupil radius is r = NA * N * dx / lambda DFT bins, and
  Circ(k) = [kx^2 + ky^2 <= r^2] (closed disk);
* shifted indices k + k_i are formed on the integers and never wrapped.
"""

import numpy as np


def pupil_radius(n, dx_um, wavelength_um, na):
    """Pupil radius in DFT bins, r = NA N dx / lambda (Eq. 1's Circ_NA)."""
    return na * n * dx_um / wavelength_um


def signed_freqs(n):
    """Signed DFT indices in FFT order: 0, 1, ..., N/2-1, -N/2, ..., -1."""
    return np.concatenate([np.arange(0, n // 2), np.arange(-(n // 2), 0)]).astype(np.int64)


def k_grid(n):
    """(ky, kx) integer grids of shape (N, N) in FFT order."""
    f = signed_freqs(n)
    ky, kx = np.meshgrid(f, f, indexing="ij")
    return ky, kx


def circ(ky, kx, r):
    """Closed disk indicator Circ(k) = [kx^2 + ky^2 <= r^2] on integer k."""
    ky = np.asarray(ky, dtype=np.int64)
    kx = np.asarray(kx, dtype=np.int64)
    return (kx * kx + ky * ky) <= r * r


def fft_index(ky, kx, n):
    """Row and column of signed frequency (ky, kx) in an FFT-ordered N x N array."""
    return np.mod(ky, n), np.mod(kx, n)


def in_range(ky, kx, n):
    """True where the signed index lies inside [-N/2, N/2)^2 (no wrap needed)."""
    h = n // 2
    return (ky >= -h) & (ky < h) & (kx >= -h) & (kx < h)
