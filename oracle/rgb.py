"""Colour image of a stained slide from three single-wavelength
reconstructions (Sec. 3.3: the method runs on each of the R, G and B channels
separately; the amplitudes of the three reconstructed fields are combined
and white balanced).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading taken (the paper does not say how it white balances): gains g_c
multiply each channel's amplitude; by default they follow the grey-world
rule, g_c = mean over channels of m / m_c with m_c the mean amplitude of
channel c over every pixel of every tile.
"""

import numpy as np


def grey_world_gains(fields_rgb):
    """fields_rgb: three complex arrays of equal shape; returns g (3,)."""
    m = np.array([np.mean(np.abs(np.asarray(f, np.complex128))) for f in fields_rgb])
    return m.mean() / m


def combine(fields_rgb, gains=None):
    """Planar colour image (..., 3, H, W) per tile: g_c |F_c|; fields_rgb are
    three complex arrays (T, H, W).  Returns (image, gains)."""
    g = grey_world_gains(fields_rgb) if gains is None else np.asarray(gains, np.float64)
    amps = [g[c] * np.abs(np.asarray(fields_rgb[c], np.complex128)) for c in range(3)]
    return np.stack(amps, axis=1), g
