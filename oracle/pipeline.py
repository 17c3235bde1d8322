"""Whole per-tile reconstruction in the order of Fig. 2: KK for every
NA-matched image (Eq. 4-7), aberration solve (Eq. 8-10), correction and
stitching, darkfield extension image by image (Eq. 11-13), upsampled output.
"""

from dataclasses import dataclass, field as dc_field

import numpy as np

from .grid import pupil_radius
from .kk import kk_field, kk_spectrum
from .aberration import estimate_pupil, PUPIL_BANDS
from .stitch import stitch_brightfield
from .darkfield import extend_darkfield
from .output import upsampled_field


@dataclass
class Geometry:
    """One tile geometry: sizes, optics and illumination vectors (kx, ky) in bins."""
    n: int
    dx_um: float
    wavelength_um: float
    na_obj: float
    k_bf: np.ndarray
    k_df: np.ndarray
    upsample: int = 2
    ridge_pupil: float = 1e-9
    ridge_darkfield: float = 1e-4
    log_floor_rel: float = 1e-6
    pupil_bands: int = 1
    extra: dict = dc_field(default_factory=dict)

    @property
    def r(self):
        return pupil_radius(self.n, self.dx_um, self.wavelength_um, self.na_obj)

    @property
    def n_bf(self):
        return len(self.k_bf)

    @property
    def n_df(self):
        return len(self.k_df)


def kk_stack(images, geom):
    """KK spectra of the NA-matched images and whether any hit the log floor."""
    floor_hit = False
    out = []
    for img, k_i in zip(images[:geom.n_bf], geom.k_bf):
        _, hit = kk_field(img, k_i, geom.log_floor_rel)
        floor_hit |= hit
        out.append(kk_spectrum(img, k_i, geom.r, geom.log_floor_rel))
    return np.stack(out), floor_hit


def reconstruct(images, geom, seed=None, zernike=None, gram="fullq", keep=False):
    """Reconstruct one tile.

    images   (n_bf + n_df, N, N) intensities: NA-matched first, then darkfield
             in processing order
    seed     optional Noll coefficients for the re-wrapped pupil solve
    zernike  optional coefficients that replace the pupil solve altogether
    Returns dict: field (fN, fN), c (15,), pupil diagnostics, darkfield info.
    """
    images = np.asarray(images, dtype=np.float64)
    r = geom.r
    spectra, floor_hit = kk_stack(images, geom)
    pupil = estimate_pupil(spectra, geom.k_bf, r, ridge=geom.ridge_pupil, seed=seed,
                           bands=PUPIL_BANDS if geom.pupil_bands else ())
    c = pupil["c"] if zernike is None else np.asarray(zernike, dtype=np.float64)
    obj_hat, known = stitch_brightfield(spectra, geom.k_bf, c, r)
    bf_hat = obj_hat.copy()
    df_info = []
    for img, k_j in zip(images[geom.n_bf:], geom.k_df):
        obj_hat, known, info = extend_darkfield(obj_hat, known, img, k_j, c, r,
                                                ridge=geom.ridge_darkfield, gram=gram)
        if not keep:
            for key in ("gram", "rhs", "b"):
                info.pop(key, None)
        df_info.append(info)
    out = {"field": upsampled_field(obj_hat, geom.upsample), "c": c, "pupil": pupil,
           "obj_hat": obj_hat, "known": known, "bf_hat": bf_hat,
           "darkfield": df_info, "log_floor_hit": floor_hit}
    if keep:
        out["spectra"] = spectra
    return out
