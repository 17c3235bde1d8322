"""Upsampled complex field from the final spectrum (Sec. 2.3: the assembled
spectrum doubles the resolution of the objective; the output is sampled
finer than the camera so that the wider spectrum fits).

Reading taken: the N x N spectrum is zero-embedded at the same signed indices
of an fN x fN grid and inverse transformed with a factor f^2, so the samples
equal the band-limited object on the dx/f grid.
"""

import numpy as np

from .grid import k_grid


def upsampled_field(obj_hat, f):
    """ifft2 of the zero-embedded spectrum on an fN x fN grid, times f^2."""
    n = obj_hat.shape[0]
    m = f * n
    big = np.zeros((m, m), dtype=np.complex128)
    ky, kx = k_grid(n)
    big[np.mod(ky, m), np.mod(kx, m)] = obj_hat
    return np.fft.ifft2(big) * float(f) ** 2
