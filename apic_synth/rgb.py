"""Three-wavelength (RGB) workload of a stained slide: the method runs once
per colour channel, each channel with its own wavelength, pupil radius,
illumination lattice and pupil.

* Channels R, G, B at 0.63, 0.52 and 0.47 um; the LEDs are physical, so every
  channel sees the same illumination NAs: 8 NA-matched LEDs at 0.25 and 8 + 8
  darkfield LEDs at 0.28 and 0.32 (half-step azimuth offset on the second
  ring).  The lattice point of each LED, and the pupil radius, scale as 1/lambda.
* Stained tissue: the smooth texture, whose optical path gives a phase scaled
  by 0.52 / lambda, under cell blobs carrying haematoxylin (nuclei) and eosin
  (cytoplasm) densities h(x), e(x); channel c transmits exp(-(h OD_H[c] +
  e OD_E[c])) with the published haematoxylin and eosin optical-density
  vectors of Ruifrok and Johnston (2001).
* Pupil: the quadratic field model at the tile's position for green, scaled
  to max |c| = 0.25 rad (inside the range where the closed-form solve's
  phase differences stay unwrapped); the same optical path difference scaled
  by 0.52 / lambda in the other channels, plus a chromatic defocus of
  +0.1 rad (R) and -0.1 rad (B) on Noll Z4.
"""

import numpy as np

from .configs import OPTICS, Workload, field_model_quadratic
from .leds import led_rings
from .objects import gaussian_smooth_periodic, minmax

CHANNELS = (("R", 0.63), ("G", 0.52), ("B", 0.47))
OD_H = np.array([0.650, 0.704, 0.286])   # haematoxylin, per R, G, B
OD_E = np.array([0.072, 0.990, 0.105])   # eosin
DEFOCUS = {"R": 0.1, "G": 0.0, "B": -0.1}


def stained_object(rng, n, channel, lam):
    """Complex transmission of one stained tile in one channel (the draws do
    not depend on the channel, so the three channels see the same tissue):
    the smooth texture (amplitude 0.85-1, optical path giving 0..pi rad at
    0.52 um, both smoothed by 2 px) with its phase scaled by 0.52 / lambda,
    times the stain transmission exp(-(h OD_H[c] + e OD_E[c])) of soft cells
    (eosin over the cell, haematoxylin over its nucleus)."""
    amp = 0.85 + 0.15 * minmax(gaussian_smooth_periodic(rng.random((n, n)), 2.0))
    psi = np.pi * minmax(gaussian_smooth_periodic(rng.standard_normal((n, n)), 2.0))
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    h = np.zeros((n, n))
    e = np.zeros((n, n))
    for _ in range(max(1, int(round(n * n / 900.0)))):
        cy, cx = rng.uniform(0, n, 2)
        ay, ax = rng.uniform(5.0, 14.0, 2)
        th = rng.uniform(0, np.pi)
        dy = (yy - cy + n / 2) % n - n / 2
        dx = (xx - cx + n / 2) % n - n / 2
        u = dx * np.cos(th) + dy * np.sin(th)
        v = -dx * np.sin(th) + dy * np.cos(th)
        q = (u / ax) ** 2 + (v / ay) ** 2
        e += rng.uniform(0.05, 0.15) * (q <= 1.0)
        h += rng.uniform(0.1, 0.3) * (q <= 0.25)
    h, e = gaussian_smooth_periodic(h, 2.0), gaussian_smooth_periodic(e, 2.0)
    k = "RGB".index(channel)
    return amp * np.exp(-(h * OD_H[k] + e * OD_E[k])) * np.exp(1j * psi * (0.52 / lam))


def config_rgb(n_tiles=4, n=128, photons=1e4):
    """One Workload per channel (R, G, B) over the same tiles (same seeds, so
    the same tissue in every channel); tile positions on a square grid of
    [-1, 1]^2."""
    side = int(np.ceil(np.sqrt(n_tiles)))
    g = np.arange(n_tiles)
    u = (g % side - (side - 1) / 2) / max(1.0, (side - 1) / 2)
    v = (g // side - (side - 1) / 2) / max(1.0, (side - 1) / 2)
    c_green, _ = field_model_quadratic(u, v, max_abs=0.25)
    out = []
    for name, lam in CHANNELS:
        rings_bf = [(0.25, 8, 0.0, True)]
        rings_df = [(0.28, 8, 0.0, False), (0.32, 8, 0.5, False)]
        kw = dict(dx_um=OPTICS["dx_um"], wavelength_um=lam, na_obj=OPTICS["na_obj"])
        c = c_green * (0.52 / lam)
        c[:, 3] += DEFOCUS[name]
        w = Workload(f"rgb-{name}", n, led_rings(n, rings_bf, **kw), led_rings(n, rings_df, **kw),
                     upsample=2, n_tiles=n_tiles, photons=photons, seed_id=60,
                     coeffs=c, positions=np.stack([u, v], axis=1), wavelength_um=lam,
                     extra={"channel": name})
        w.obj_fn = (lambda rng, nn, _c=name, _l=lam: stained_object(rng, nn, _c, _l))
        out.append(w)
    return out
