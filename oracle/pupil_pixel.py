"""Pupil-aberration solve of Eq. 10 with one unknown per pupil pixel (the
paper's own formulation: phi is the flattened pupil-plane phase, and each row
of D takes four of its samples).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Unknowns: phi(k) at every integer k with kx^2 + ky^2 <= r^2, numbered in
raster order (ky ascending, then kx ascending).  Rows, phase differences and
weights are those of the Zernike-basis solve (same pairs, same K, beta = arg
of s_i(K) conj(s_l(K)), w = |s_i(K) s_l(K)|); the row operator is
phi(K+K_i) - phi(K+K_l) - phi(K_i) + phi(K_l) with coincident samples merged.

Readings taken (the paper names no solver):
* phi is the minimum-norm weighted least-squares solution of D phi = beta
  (weights w): the solution of D^T W D phi = D^T W beta with no component in
  the null space of D.  That null space holds piston, tip and tilt, and in
  some LED layouts more: when every LED difference K_i - K_l lies on a
  sublattice of the integer grid, functions periodic on that sublattice
  (for instance (-1)^(kx + ky) when all kx + ky are even) cancel in every row;
* the pixel phase is summarised by its least-squares fit of Noll Z_1..Z_15
  over the pupil pixels, reported as c_4..c_15 (c_1..c_3 are the gauge and
  reported as 0).
Here the normal matrix is formed densely and inverted on its range through its
eigendecomposition (eigenvalues under 1e-10 of the largest count as null).
For pupils too large for a dense normal matrix (512 px tiles: about 30,000
pixels) the same minimum-norm solution is taken by LSQR on the weighted rows
sqrt(w) D phi = sqrt(w) beta started from zero (scipy's LSQR, a library
primitive: its iterates stay in the range of D^T, so it ends at the
minimum-norm least-squares solution); the tests pin the two routes to each
other on the smaller geometries.
"""

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .aberration import pupil_pairs
from .grid import fft_index
from .zernike import zernike


def pupil_pixels(n, r):
    """(ky, kx) of the pupil pixels in raster order, and an (N, N) index map in
    centred layout (row ky + N/2, column kx + N/2; -1 outside the pupil)."""
    h = n // 2
    ky, kx = np.meshgrid(np.arange(-h, h), np.arange(-h, h), indexing="ij")
    inside = kx * kx + ky * ky <= r * r
    idx = -np.ones((n, n), np.int64)
    idx[inside] = np.arange(int(inside.sum()))
    return ky[inside], kx[inside], idx


def pixel_system(spectra, k_bf, r):
    """Sparse D (rows x N_p), beta and w of Eq. 10 on the pupil pixels."""
    n = spectra.shape[-1]
    h = n // 2
    k_bf = np.asarray(k_bf, dtype=np.int64)
    pky, pkx, idx = pupil_pixels(n, r)
    rows, cols, vals, betas, ws = [], [], [], [], []
    m = 0
    for i, l, K_y, K_x in pupil_pairs(n, k_bf, r):
        yy, xx = fft_index(K_y, K_x, n)
        z = spectra[i][yy, xx] * np.conj(spectra[l][yy, xx])
        betas.append(np.arctan2(z.imag, z.real))
        ws.append(np.abs(z))
        ki, kl = k_bf[i], k_bf[l]
        a = idx[K_y + ki[1] + h, K_x + ki[0] + h]
        b = idx[K_y + kl[1] + h, K_x + kl[0] + h]
        c = idx[ki[1] + h, ki[0] + h]
        d = idx[kl[1] + h, kl[0] + h]
        assert np.all(a >= 0) and np.all(b >= 0) and c >= 0 and d >= 0
        R = np.arange(m, m + len(K_y))
        for col, v in ((a, 1.0), (b, -1.0), (np.full(len(R), c), -1.0), (np.full(len(R), d), 1.0)):
            rows.append(R)
            cols.append(col)
            vals.append(np.full(len(R), v))
        m += len(K_y)
    D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, len(pky)))  # duplicate entries are summed (merged samples)
    return D, np.concatenate(betas), np.concatenate(ws), (pky, pkx)


def solve_pixel_pupil(spectra, k_bf, r, null_rel=1e-10, method="eig", tol=1e-13,
                      iter_lim=200000):
    """Eq. 10 on the pupil pixels.  Returns dict with phi (N_p,), the pixel
    coordinates, phi_map (N, N) in FFT order (0 outside the pupil), c (15,)
    the Zernike summary and the null-space dimension found (eig) or the LSQR
    iterations taken (lsqr, where null_dim is None)."""
    n = spectra.shape[-1]
    D, beta, w, (pky, pkx) = pixel_system(spectra, k_bf, r)
    null_dim, iters = None, None
    if method == "eig":
        Dw = D.multiply(w[:, None]).tocsr()
        A = (D.T @ Dw).toarray()
        rhs = D.T @ (w * beta)
        ev, U = scipy.linalg.eigh(A)
        keep = ev > null_rel * ev.max()
        phi = U[:, keep] @ ((U[:, keep].T @ rhs) / ev[keep])
        null_dim = int((~keep).sum())
    elif method == "lsqr":
        sw = np.sqrt(w)
        out = spla.lsqr(D.multiply(sw[:, None]).tocsr(), sw * beta, atol=tol, btol=tol,
                        conlim=1e12, iter_lim=iter_lim)
        phi, iters = out[0], int(out[2])
    else:
        raise ValueError(method)
    phi_map = np.zeros((n, n))
    yy, xx = fft_index(pky, pkx, n)
    phi_map[yy, xx] = phi
    return {"phi": phi, "ky": pky, "kx": pkx, "phi_map": phi_map,
            "c": zernike_summary(phi, pky, pkx, r), "rows": D.shape[0],
            "null_dim": null_dim, "iters": iters}


def zernike_summary(phi, pky, pkx, r):
    """Least-squares fit of Noll Z_1..Z_15 to phi over the pupil pixels;
    returns c (15,) with c_1..c_3 set to 0."""
    Z = np.stack([zernike(j, pky, pkx, r) for j in range(1, 16)], axis=1)
    c, *_ = np.linalg.lstsq(Z, phi, rcond=None)
    c[:3] = 0.0
    return c
