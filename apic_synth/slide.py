"""Slide-scale stream workload (whole-slide scanning, stands in for the
paper's slide experiments).

* Slide 76 x 25 mm cut into 512 px tiles of 0.4 um pixels: a 122 x 371 grid,
  scanned in raster order (row by row).
* Tissue mask: white noise (default_rng([4, 0, 0])) smoothed by a Gaussian of
  2 mm, thresholded at its 70th percentile, so 30% of the tiles hold tissue;
  only those are scanned.
* Content comes from a pool of pre-generated tiles that the scanned positions
  cycle through: tissue tiles (soft elliptical cells, ``object_blobs``) and a
  few near-empty glass tiles (``object_background``) standing for patches of a
  scanned field of view that fall on glass.  Each pool tile keeps its own
  field position (u, v) in [-1, 1]^2 (default_rng([4, 2, 0])) and the pupil
  of the scaled quadratic field model there (max |c| 1.5 rad over a 64 x 64
  grid).  16 NA-matched images (ring at NA 0.25), 32 darkfield (rings at NA
  0.30 and 0.38), Poisson noise at 1e4 photons.
"""

import numpy as np
from scipy.ndimage import gaussian_filter

from .configs import OPTICS, Workload
from .leds import led_rings
from .objects import object_blobs
from .surrogate_set import field_coeffs, pupil_at

N = 512


def slide_grid(width_mm=76.0, height_mm=25.0, n=N, dx_um=OPTICS["dx_um"]):
    """(rows, cols) of whole tiles on the slide."""
    tile_um = n * dx_um
    return int(height_mm * 1000 // tile_um), int(width_mm * 1000 // tile_um)


def slide_mask(rows=None, cols=None, sigma_mm=2.0, tissue_frac=0.30, n=N,
               dx_um=OPTICS["dx_um"]):
    """Boolean (rows, cols) tissue mask; True = tissue."""
    if rows is None or cols is None:
        rows, cols = slide_grid(n=n, dx_um=dx_um)
    rng = np.random.default_rng([4, 0, 0])
    sigma_tiles = sigma_mm * 1000.0 / (n * dx_um)
    sm = gaussian_filter(rng.standard_normal((rows, cols)), sigma_tiles, mode="reflect")
    return sm > np.quantile(sm, 1.0 - tissue_frac)


def pool_workload(p_tissue=16, p_glass=4, photons=1e4, max_abs=1.5):
    """The pool as one Workload: tissue tiles first, then glass tiles."""
    n = N
    leds_bf = led_rings(n, [(0.25, 16, 0.0, True)])
    leds_df = led_rings(n, [(0.30, 16, 0.0, False), (0.38, 16, 0.5, False)])
    p = p_tissue + p_glass
    uv = np.random.default_rng([4, 2, 0]).uniform(-1.0, 1.0, (p, 2))
    coeffs = pupil_at(field_coeffs(max_abs), uv)
    glass = np.zeros(p, bool)
    glass[p_tissue:] = True
    return Workload("slide-pool", n, leds_bf, leds_df, upsample=2, n_tiles=p, photons=photons,
                    seed_id=4, obj_fn=object_blobs, coeffs=coeffs, positions=uv,
                    extra={"background": glass})


def scan_order(mask, n_scanned, p_tissue, p_glass, glass_frac=0.15):
    """Raster indices of the first ``n_scanned`` tissue tiles of the mask and,
    for each, the pool tile it shows: glass with probability ``glass_frac``
    (default_rng([4, 2, 1])), else the next tissue tile, cycling."""
    idx = np.flatnonzero(mask.ravel())[:n_scanned]
    rng = np.random.default_rng([4, 2, 1])
    is_glass = rng.uniform(size=len(idx)) < glass_frac if p_glass else np.zeros(len(idx), bool)
    src = np.empty(len(idx), np.int64)
    ti = gi = 0
    for k in range(len(idx)):
        if is_glass[k]:
            src[k] = p_tissue + gi % p_glass
            gi += 1
        else:
            src[k] = ti % p_tissue
            ti += 1
    return idx, src
