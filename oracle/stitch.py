"""Aberration correction and brightfield stitching (Sec. 2.3, the text after
Eq. 10 and the caption of Fig. 2).

After Eq. 10 is solved, each KK spectrum is corrected for the pupil phase and
the corrected spectra are assembled into one spectrum of twice the objective's
bandwidth.  Eq. 7 says that image i carries exp(j[phi(k + k_i) - phi(k_i)]) on
its support, so correction divides that factor out.

Reading taken: the corrected spectra are combined by the plain average over the NA-matched
images that cover each frequency; the known set is where at least one covers.
"""

import numpy as np

from .grid import k_grid, circ
from .zernike import pupil_phase


def stitch_brightfield(spectra, k_bf, c, r):
    """Corrected, averaged brightfield spectrum and its known set.

    Returns (O_hat complex (N, N), known bool (N, N)).
    """
    n = spectra.shape[-1]
    ky, kx = k_grid(n)
    acc = np.zeros((n, n), dtype=np.complex128)
    count = np.zeros((n, n))
    for s_i, k_i in zip(spectra, np.asarray(k_bf, dtype=np.int64)):
        qy, qx = ky + k_i[1], kx + k_i[0]
        support = circ(qy, qx, r)
        phase = pupil_phase(c, qy, qx, r) - pupil_phase(c, k_i[1], k_i[0], r)
        acc += np.where(support, s_i * np.exp(-1j * phase), 0.0)
        count += support
    known = count > 0
    obj_hat = np.where(known, acc / np.maximum(count, 1.0), 0.0)
    return obj_hat, known
