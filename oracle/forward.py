"""The oracle's own image-formation model (Sec. 2.2, Eq. 1-2; Eq. 3).

Eq. 1 puts the object spectrum, shifted by the illumination vector k_i, behind
the coherent transfer function Circ_NA(k) exp(j phi(k)); Eq. 2 records the
squared modulus of its inverse transform.  Eq. 3 shows that the image does not
change if the whole spectrum is moved back by k_i, so the oracle forms the
image in that shifted frame,

    S'_i(k) = O_hat(k) Circ(k + k_i) exp(j phi(k + k_i)),   I_i = |ifft2 S'_i|^2,

which equals Eq. 1-2 for integer k_i and needs no wrap of the object spectrum.
"""

import numpy as np

from .grid import k_grid, circ
from .zernike import pupil_phase


def shifted_spectrum(obj_hat, k_i, c, r):
    """S'_i(k) for one illumination vector k_i = (kx, ky) (Eq. 1 and Eq. 3)."""
    n = obj_hat.shape[0]
    ky, kx = k_grid(n)
    qy = ky + int(k_i[1])
    qx = kx + int(k_i[0])
    support = circ(qy, qx, r)
    phase = np.where(support, pupil_phase(c, qy, qx, r), 0.0)
    return np.where(support, obj_hat * np.exp(1j * phase), 0.0)


def forward_images(obj, k_list, c, r):
    """Noise-free intensities I_i (Eq. 2) for every k_i in ``k_list``.

    obj    complex (N, N) object transmission O(x)
    k_list (n, 2) integer illumination vectors (kx, ky) in DFT bins
    c      Noll coefficients of the true pupil phase (c[0] is j = 1)
    r      pupil radius in bins
    Returns float64 (n, N, N).
    """
    obj_hat = np.fft.fft2(np.asarray(obj, dtype=np.complex128))
    out = []
    for k_i in np.asarray(k_list, dtype=np.int64):
        s = np.fft.ifft2(shifted_spectrum(obj_hat, k_i, c, r))
        out.append(np.abs(s) ** 2)
    return np.stack(out)
