"""Synthetic thin-sample transmissions O(x) = a(x) exp(j psi(x)).

All filtering is periodic (the tiles are periodic), done by multiplying the DFT
with the transform of a Gaussian of standard deviation sigma pixels.
"""

import numpy as np


def gaussian_smooth_periodic(x, sigma):
    """Periodic Gaussian smoothing of a real (N, N) array."""
    n0, n1 = x.shape
    fy = np.fft.fftfreq(n0)[:, None]
    fx = np.fft.fftfreq(n1)[None, :]
    h = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * (fy ** 2 + fx ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(x) * h))


def minmax(x):
    """Rescale to [0, 1]."""
    lo, hi = float(x.min()), float(x.max())
    return (x - lo) / (hi - lo) if hi > lo else np.zeros_like(x)


def object_smooth(rng, n, sigma=2.0):
    """Amplitude 0.85-1.0 and phase 0..pi, both smoothed by a sigma-px Gaussian."""
    amp = 0.85 + 0.15 * minmax(gaussian_smooth_periodic(rng.random((n, n)), sigma))
    psi = np.pi * minmax(gaussian_smooth_periodic(rng.standard_normal((n, n)), sigma))
    return amp * np.exp(1j * psi)


def object_weak(rng, n, eps, sigma=2.0):
    """Weak object 1 + eps * o with o a smoothed complex noise of unit max."""
    o = (gaussian_smooth_periodic(rng.standard_normal((n, n)), sigma)
         + 1j * gaussian_smooth_periodic(rng.standard_normal((n, n)), sigma))
    return 1.0 + eps * o / np.abs(o).max()


def object_background(rng, n, sigma=2.0):
    """Near-empty glass: amplitude in [0.99, 1], phase std U(0.005, 0.02) rad."""
    amp = 0.99 + 0.01 * minmax(gaussian_smooth_periodic(rng.random((n, n)), sigma))
    psi = gaussian_smooth_periodic(rng.standard_normal((n, n)), sigma)
    psi = psi / max(psi.std(), 1e-12) * rng.uniform(0.005, 0.02)
    return amp * np.exp(1j * psi)


def object_blobs(rng, n, sigma_edge=1.5, px_per_blob=1500.0):
    """Tissue-like object: soft elliptical cells with phase 0.5-2 rad on a smooth
    amplitude."""
    amp = 0.85 + 0.15 * minmax(gaussian_smooth_periodic(rng.random((n, n)), 2.0))
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    psi = np.zeros((n, n))
    count = max(1, int(round(n * n / px_per_blob)))
    for _ in range(count):
        cy, cx = rng.uniform(0, n, size=2)
        ay, ax = rng.uniform(6.0, 20.0, size=2)
        th = rng.uniform(0, np.pi)
        dy = (yy - cy + n / 2) % n - n / 2
        dx = (xx - cx + n / 2) % n - n / 2
        u = dx * np.cos(th) + dy * np.sin(th)
        v = -dx * np.sin(th) + dy * np.cos(th)
        inside = ((u / ax) ** 2 + (v / ay) ** 2) <= 1.0
        psi += rng.uniform(0.5, 2.0) * inside
    psi = gaussian_smooth_periodic(psi, sigma_edge)
    return amp * np.exp(1j * psi)
