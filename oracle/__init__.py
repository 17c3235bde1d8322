"""FP64 CPU oracle for the per-tile closed-form APIC reconstruction.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
NumPy/SciPy implementation of what the GPU path computes, written step by step
from the paper (Zhao, Zhou, Lin, Cao, Yang, "Efficient, gigapixel-scale,
aberration-free whole slide scanner using angular ptychographic imaging with
closed-form solution", arXiv 2407.20469):

  forward model ........ Sec. 2.2, Eq. 1-3            (forward.py)
  Kramers-Kronig ....... Sec. 2.3, Eq. 4-7            (kk.py)
  aberration solve ..... Sec. 2.3, Eq. 8-10           (aberration.py)
  pixel-domain Eq. 10 .. Sec. 2.3, Eq. 10 per pixel   (pupil_pixel.py)
  correction + stitch .. Sec. 2.3 text after Eq. 10   (stitch.py)
  darkfield extension .. Sec. 2.3, Eq. 11-13          (darkfield.py)
  upsampled output ..... Sec. 2.3, end of brightfield part (output.py)
  background test ...... Sec. 3.2, variance threshold (background.py)
  patch assembly ....... Sec. 2.5, overlap blending  (assemble.py)
  colour combination ... Sec. 3.3, RGB channels      (rgb.py)
  surrogate MLP twin ... not in the paper             (mlp.py)
  surrogate fallback ... not in the paper; Eq. 10 judges (fallback.py)

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or execute anything in this package.  The product path
(``paper_2407_20469_amd``) never imports it and shares no code with it; the
only module both sides use is ``apic_synth`` (seeded inputs, no method
arithmetic).

Every function computes in float64 / complex128.  Where the paper is silent or
garbled, the reading taken is stated in the docstring of the function that
takes it.

Parity pins live in ``tests/test_oracle_*.py``; each oracle function is pinned
against closed forms, brute force, invariants or the paper's printed numbers.
"""

from .grid import k_grid, circ, pupil_radius, fft_index
from .zernike import noll_nm, zernike, pupil_phase
from .forward import forward_images
from .kk import kk_field, kk_spectrum
from .aberration import aberration_sums, solve_aberration, estimate_pupil, pupil_pairs
from .stitch import stitch_brightfield
from .darkfield import darkfield_sets, extend_darkfield
from .output import upsampled_field
from .background import background_stat, is_background
from .pupil_pixel import solve_pixel_pupil
from .pipeline import Geometry, reconstruct

__all__ = [
    "k_grid", "circ", "pupil_radius", "fft_index",
    "noll_nm", "zernike", "pupil_phase",
    "forward_images", "kk_field", "kk_spectrum",
    "aberration_sums", "solve_aberration", "estimate_pupil", "pupil_pairs",
    "stitch_brightfield", "darkfield_sets", "extend_darkfield",
    "upsampled_field", "Geometry", "reconstruct",
]
