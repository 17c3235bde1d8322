"""Darkfield spectrum extension (Sec. 2.3, Eq. 11-13 and the paragraph after).

Eq. 11 splits a darkfield image into the field of the already-known part of its
spectrum (P) and of the unknown part (U); Eq. 12 is its transform, a sum of
four correlations.  Eq. 13 keeps the frequencies where only the cross term
P-hat * U-hat survives, which is linear in the unknown U-hat; the paragraph
after Eq. 13 writes that correlation as a matrix C (M equations, one per
frequency of Q, times N_u unknowns) and solves the linear system.

With NumPy's DFT normalisation, fft2(P conj(U))(k) = N^-2 sum_u P_hat(u+k)
conj(U_hat(u)), so after conjugation

    conj(fft2(I_j)(k) - fft2(|P|^2)(k)) = sum_u C[k, u] U_hat(u),
    C[k, u] = conj(P_hat(u + k)) / N^2,   k in Q,  u in U.

Readings taken:
* the darkfield images are used one after another in the order given; the
  unknowns solved by one image are known for all later ones (never revisited);
  an image whose unknown set is empty is skipped;
* Q removes both the U-U autocorrelation support and the mirrored cross term
  support U - P (Eq. 13 is false on the latter);
* the known spectrum carries the pupil phase of the darkfield image, and the
  solved spectrum has it divided out (Sec. 2.3 applies the estimated aberration
  to the spectra of both image types);
* the system is solved as Tikhonov least squares through the normal equations,
  ridge lambda * tr(C^H C) / N_u, by FP64 Cholesky.
"""

import numpy as np
import scipy.linalg

from .grid import k_grid, circ, fft_index, in_range
from .zernike import pupil_phase

ROW_CHUNK = 2048


def coords_of(mask):
    """Signed (ky, kx) of the True entries of an FFT-ordered mask, in row-major
    FFT-index order."""
    n = mask.shape[0]
    ky, kx = k_grid(n)
    return np.stack([ky[mask], kx[mask]], axis=1)


def minkowski_diff(a, b, n):
    """Boolean grid over [-n, n]^2 (offset n) of the set {p - q : p in a, q in b},
    looping over the smaller of the two sets."""
    grid = np.zeros((2 * n + 1, 2 * n + 1), dtype=bool)
    if len(b) <= len(a):
        for qy, qx in b:
            grid[a[:, 0] - qy + n, a[:, 1] - qx + n] = True
    else:
        for py, px in a:
            grid[py - b[:, 0] + n, px - b[:, 1] + n] = True
    return grid


def darkfield_sets(n, k_j, known, r):
    """P, U, Q, E of one darkfield image as coordinate arrays.

    D = Circ(k + k_j); P = D & known; U = D & ~known;
    Q = (P - U) minus ((U - U) or (U - P)); E = (P - U) and ((U - U) or (U - P)).
    Q and E are returned in row-major FFT-index order.
    """
    ky, kx = k_grid(n)
    disk = circ(ky + int(k_j[1]), kx + int(k_j[0]), r)
    p_mask = disk & known
    u_mask = disk & ~known
    p = coords_of(p_mask)
    u = coords_of(u_mask)
    if len(u) == 0:
        return {"P": p, "U": u, "Q": np.zeros((0, 2), np.int64), "E": np.zeros((0, 2), np.int64),
                "P_mask": p_mask, "U_mask": u_mask}
    pu = minkowski_diff(p, u, n)
    excl = minkowski_diff(u, u, n) | minkowski_diff(u, p, n)
    off = np.arange(-n, n + 1)
    gy, gx = np.meshgrid(off, off, indexing="ij")

    def ordered(sel):
        yy, xx = gy[sel], gx[sel]
        assert np.all(in_range(yy, xx, n)), "difference set wraps the DFT grid"
        order = np.lexsort((np.mod(xx, n), np.mod(yy, n)))
        return np.stack([yy[order], xx[order]], axis=1)

    return {"P": p, "U": u, "Q": ordered(pu & ~excl), "E": ordered(pu & excl),
            "P_mask": p_mask, "U_mask": u_mask}


def gather_signed(arr, ky, kx):
    """arr at signed (ky, kx); zero where the index falls outside the grid."""
    n = arr.shape[0]
    ok = in_range(ky, kx, n)
    yy, xx = fft_index(np.where(ok, ky, 0), np.where(ok, kx, 0), n)
    return np.where(ok, arr[yy, xx], 0.0)


def padded_spectrum(p_hat):
    """P_hat at its signed positions on a 2N x 2N zero grid: indexing it at
    (ky mod 2N, kx mod 2N) for any ky, kx in [-N, N) gives P_hat(ky, kx)
    inside [-N/2, N/2)^2 and 0 outside, as ``gather_signed`` does."""
    n = p_hat.shape[0]
    ky, kx = k_grid(n)
    out = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    out[np.mod(ky, 2 * n), np.mod(kx, 2 * n)] = p_hat
    return out


def conv_matrix(p_hat, q, u, padded=None):
    """C[k, u] = conj(P_hat(u + k)) / N^2 for rows k in q, columns u in u
    (every u + k lies in [-N, N)); ``padded`` is ``padded_spectrum(p_hat)``
    when the caller has it."""
    n = p_hat.shape[0]
    pad = padded_spectrum(p_hat) if padded is None else padded
    ky = np.mod(q[:, 0][:, None] + u[:, 0][None, :], 2 * n)
    kx = np.mod(q[:, 1][:, None] + u[:, 1][None, :], 2 * n)
    return np.conj(pad[ky, kx]) / float(n) ** 2


def normal_equations_fullq(p_hat, q, u, b):
    """G = C^H C and C^H b, C built row chunk by row chunk."""
    nu = len(u)
    g = np.zeros((nu, nu), dtype=np.complex128)
    v = np.zeros(nu, dtype=np.complex128)
    pad = padded_spectrum(p_hat)
    for s in range(0, len(q), ROW_CHUNK):
        c = conv_matrix(p_hat, q[s:s + ROW_CHUNK], u, pad)
        g += c.conj().T @ c
        v += c.conj().T @ b[s:s + ROW_CHUNK]
    return g, v


def autocorrelation(p_hat, p, d):
    """R(d) = sum_{p in P} P_hat(p) conj(P_hat(p + d)) for each row of d."""
    vals = gather_signed(p_hat, p[:, 0], p[:, 1])
    out = np.zeros(len(d), dtype=np.complex128)
    for idx, (dy, dx) in enumerate(d):
        out[idx] = np.sum(vals * np.conj(gather_signed(p_hat, p[:, 0] + dy, p[:, 1] + dx)))
    return out


def autocorrelation_grid(p_hat):
    """R(d) = sum_p P_hat(p) conj(P_hat(p + d)) for every d in [-N, N)^2.

    The spectrum is placed at its signed positions on a 2N x 2N grid, where
    no product of the linear sum wraps, and the correlation is taken by FFT:
    with a = conj(P_hat) on that grid, ifft2(|fft2(a)|^2)(d) = sum_p conj(a(p))
    a(p + d) = R(d).  Returned as a (2N, 2N) array indexed by d mod 2N."""
    n = p_hat.shape[0]
    ky, kx = k_grid(n)
    a = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    a[np.mod(ky, 2 * n), np.mod(kx, 2 * n)] = np.conj(p_hat)
    fa = np.fft.fft2(a)
    return np.fft.ifft2(np.abs(fa) ** 2)


def rhs_by_correlation(p_hat, q, u, b):
    """C^H b = N^-2 sum_{k in Q} P_hat(u + k) b(k) for every u in U, as a
    linear cross-correlation on a 2N x 2N grid (every u + k lies in
    [-N, N - 2], so nothing wraps): with x = conj(b) placed at Q,
    ifft2(conj(fft2(x)) fft2(P_hat))(u) = sum_k b(k) P_hat(k + u)."""
    n = p_hat.shape[0]
    ky, kx = k_grid(n)
    grid_p = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    grid_p[np.mod(ky, 2 * n), np.mod(kx, 2 * n)] = p_hat
    grid_b = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    grid_b[np.mod(q[:, 0], 2 * n), np.mod(q[:, 1], 2 * n)] = np.conj(b)
    corr = np.fft.ifft2(np.conj(np.fft.fft2(grid_b)) * np.fft.fft2(grid_p))
    return corr[np.mod(u[:, 0], 2 * n), np.mod(u[:, 1], 2 * n)] / float(n) ** 2


def gram_t_minus_e(p_hat, sets):
    """The same gram as ``normal_equations_fullq`` through the identity
    G[u, u'] = R(u' - u)/N^4 - sum_{k in E} P_hat(u+k) conj(P_hat(u'+k))/N^4,
    where the first term sums over every k (all of P - U) and E = (P - U) - Q.
    R comes from ``autocorrelation_grid``; the E-sum is C restricted to the
    rows of E, built chunk by chunk."""
    n = p_hat.shape[0]
    u, e = sets["U"], sets["E"]
    rgrid = autocorrelation_grid(p_hat)
    dy = np.mod(u[None, :, 0] - u[:, None, 0], 2 * n)   # (u' - u) for [u, u']
    dx = np.mod(u[None, :, 1] - u[:, None, 1], 2 * n)
    g = rgrid[dy, dx] / float(n) ** 4
    del dy, dx
    pad = padded_spectrum(p_hat)
    for s in range(0, len(e), ROW_CHUNK):
        ce = conv_matrix(p_hat, e[s:s + ROW_CHUNK], u, pad)
        g -= ce.conj().T @ ce
    return g


def extend_darkfield(obj_hat, known, intensity, k_j, c, r, ridge=1e-4, gram="fullq"):
    """Solve one darkfield image (Eq. 11-13); returns updated (O_hat, known, info)."""
    n = obj_hat.shape[0]
    sets = darkfield_sets(n, k_j, known, r)
    info = {"n_u": len(sets["U"]), "m": len(sets["Q"]), "skipped": len(sets["U"]) == 0}
    if info["skipped"]:
        return obj_hat, known, info
    ky, kx = k_grid(n)
    qy, qx = ky + int(k_j[1]), kx + int(k_j[0])
    phase = pupil_phase(c, qy, qx, r)
    p_hat = np.where(sets["P_mask"], obj_hat * np.exp(1j * phase), 0.0)
    f_img = np.fft.fft2(np.asarray(intensity, dtype=np.float64))
    f_pp = np.fft.fft2(np.abs(np.fft.ifft2(p_hat)) ** 2)
    qq = sets["Q"]
    yy, xx = fft_index(qq[:, 0], qq[:, 1], n)
    b = np.conj(f_img[yy, xx] - f_pp[yy, xx])
    if gram == "t-e":
        g = gram_t_minus_e(p_hat, sets)
        v = rhs_by_correlation(p_hat, qq, sets["U"], b)
    else:
        g, v = normal_equations_fullq(p_hat, qq, sets["U"], b)
    lam = ridge * np.trace(g).real / len(sets["U"])
    cf = scipy.linalg.cho_factor(g + lam * np.eye(len(sets["U"])), lower=True)
    x = scipy.linalg.cho_solve(cf, v)
    u = sets["U"]
    uy, ux = fft_index(u[:, 0], u[:, 1], n)
    new_hat = obj_hat.copy()
    new_hat[uy, ux] = x * np.exp(-1j * phase[uy, ux])
    new_known = known | sets["U_mask"]
    info.update({"x": x, "gram": g, "rhs": v, "b": b})
    return new_hat, new_known, info
