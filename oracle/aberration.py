"""Pupil-aberration solve from phase differences of overlapping KK spectra
(Sec. 2.3, Eq. 8-10), written in the Zernike basis.

Eq. 8 defines the overlap S_il of the supports of images i and l.  Eq. 9 shows
that inside it the phase difference of the two recovered spectra no longer
depends on the object: it equals phi(K + K_i) - phi(K + K_l) - (theta_i -
theta_l).  Eq. 10 stacks these relations over every overlapping pair into one
linear system D phi = beta_Delta.

Readings taken:
* Eq. 10's row operator is phi(K+K_i) - phi(K+K_l) - phi(K_i) + phi(K_l)
  (the printed "D_il - D^0_ij" is read as D^0_il);
* the unknown is phi = sum_{j=4..15} c_j Z_j (piston/tip/tilt are in the
  operator's null space and fixed to 0);
* every pair i < l whose overlap minus K = 0 is not empty is used; K = 0 is
  dropped (its row is 0 = 0 after KK fixes the DC phase);
* beta = atan2(Im z, Re z) of z = s_i(K) conj(s_l(K)), and each row carries
  weight w = |z|;
* least squares by normal equations with a ridge mu * tr(A) / 12, FP64
  Cholesky;
* optional seeded variant: beta is re-wrapped around a seed c0, one pass;
* coarse-to-fine continuation (the default; the paper does not discuss the
  wrap of beta): the relation is first solved on the rows with |K| <= f r for
  growing f (0.05, 0.1, 0.2, 0.4, 0.8, 1.6), each band's solution being the
  seed about which the next band re-wraps beta, and last on every row seeded
  by the last band.  Near K = 0 the row operator is about K times a gradient
  difference of the pupil phase, so the low-|K| rows stay unwrapped however
  large the aberration, and every later band only has to add a correction
  smaller than pi.  A band holding fewer than MIN_BAND_ROWS rows (32, above
  the 12 unknowns; the band ridge below covers what its rows leave
  unconstrained) is skipped.  The first band solved must be small enough that
  its rows do not wrap: on 128 px tiles with 8 NA-matched LEDs the two
  smallest bands hold 40 and 168 rows.
  The band solves carry a strong ridge (PUPIL_BAND_RIDGE tr(A) / 12): the
  low-|K| rows leave some directions of c nearly unconstrained, and the ridge
  keeps the band's increment there near zero instead of fitting noise, which
  the next band's re-wrap would then amplify; the final pass keeps the
  ordinary ridge.  With a caller's seed the one seeded pass is used instead.
"""

import numpy as np
import scipy.linalg

from .grid import k_grid, circ, fft_index
from .zernike import zernike, SOLVED

N_FEATURE_ANGLE = 8
N_FEATURE_BAND = 4
N_FEATURES = N_FEATURE_ANGLE * N_FEATURE_BAND
PUPIL_BANDS = (0.05, 0.1, 0.2, 0.4, 0.8, 1.6)
MIN_BAND_ROWS = 32
PUPIL_BAND_RIDGE = 0.1


def pupil_pairs(n, k_bf, r):
    """Overlapping pairs (Eq. 8): list of (i, l, ky, kx) with K != 0, i < l."""
    ky, kx = k_grid(n)
    k_bf = np.asarray(k_bf, dtype=np.int64)
    nonzero = (ky != 0) | (kx != 0)
    pairs = []
    for i in range(len(k_bf)):
        si = circ(ky + k_bf[i, 1], kx + k_bf[i, 0], r)
        for l in range(i + 1, len(k_bf)):
            sl = circ(ky + k_bf[l, 1], kx + k_bf[l, 0], r)
            sel = si & sl & nonzero
            if sel.any():
                pairs.append((i, l, ky[sel], kx[sel]))
    return pairs


def row_operator(K_y, K_x, k_i, k_l, r):
    """Rows of Eq. 10 in the Zernike basis, one column per j in 4..15."""
    cols = []
    for j in SOLVED:
        cols.append(zernike(j, K_y + k_i[1], K_x + k_i[0], r)
                    - zernike(j, K_y + k_l[1], K_x + k_l[0], r)
                    - zernike(j, k_i[1], k_i[0], r)
                    + zernike(j, k_l[1], k_l[0], r))
    return np.stack(cols, axis=1)


def feature_cell(k_i, k_l, K_y, K_x, r):
    """Surrogate feature cell of each row: angle bin of (k_i, k_l) x |K|/(2r) band."""
    ki = np.asarray(k_i, dtype=np.float64)
    kl = np.asarray(k_l, dtype=np.float64)
    cosang = np.dot(ki, kl) / (np.linalg.norm(ki) * np.linalg.norm(kl))
    ang = np.arccos(np.clip(cosang, -1.0, 1.0))
    abin = int(np.clip(np.ceil(ang / (np.pi / N_FEATURE_ANGLE) - 1e-9) - 1, 0, N_FEATURE_ANGLE - 1))
    rho = np.hypot(K_x.astype(np.float64), K_y.astype(np.float64)) / (2.0 * r)
    band = np.clip(np.ceil(N_FEATURE_BAND * rho - 1e-9) - 1, 0, N_FEATURE_BAND - 1).astype(np.int64)
    return abin * N_FEATURE_BAND + band


def wrap(x):
    """Wrap a phase to [-pi, pi] by removing the nearest multiple of 2 pi."""
    return x - 2.0 * np.pi * np.round(x / (2.0 * np.pi))


def aberration_sums(spectra, k_bf, r, seed=None, k_max=None):
    """Normal-equation sums of Eq. 10 over all overlapping pairs.

    spectra  complex (n_bf, N, N) KK spectra in FFT order
    seed     optional Noll coefficients c0 (15,) for the re-wrapped variant
    k_max    optional: only the rows with |K| <= k_max
    Returns dict with A (12x12), b (12), sbb, sw, rows, and the 32 per-cell
    weight sums used as surrogate features.
    """
    n = spectra.shape[-1]
    k_bf = np.asarray(k_bf, dtype=np.int64)
    A = np.zeros((len(SOLVED), len(SOLVED)))
    b = np.zeros(len(SOLVED))
    sbb = 0.0
    sw = 0.0
    rows = 0
    cells = np.zeros(N_FEATURES)
    c0 = None if seed is None else np.asarray(seed, dtype=np.float64)[3:15]
    for i, l, K_y, K_x in pupil_pairs(n, k_bf, r):
        if k_max is not None:
            sel = K_x.astype(np.float64) ** 2 + K_y.astype(np.float64) ** 2 <= k_max * k_max
            K_y, K_x = K_y[sel], K_x[sel]
            if len(K_y) == 0:
                continue
        yy, xx = fft_index(K_y, K_x, n)
        z = spectra[i][yy, xx] * np.conj(spectra[l][yy, xx])
        beta = np.arctan2(z.imag, z.real)
        w = np.abs(z)
        a = row_operator(K_y, K_x, k_bf[i], k_bf[l], r)
        if c0 is not None:
            beta = wrap(beta - a @ c0)
        A += (a * w[:, None]).T @ a
        b += a.T @ (w * beta)
        sbb += float(np.sum(w * beta * beta))
        sw += float(np.sum(w))
        rows += len(w)
        np.add.at(cells, feature_cell(k_bf[i], k_bf[l], K_y, K_x, r), w)
    return {"A": A, "b": b, "sbb": sbb, "sw": sw, "rows": rows,
            "features": np.log1p(cells / float(n) ** 4)}


def solve_aberration(sums, ridge=1e-9, seed=None):
    """c_J = (A + ridge tr(A)/12 I)^-1 b by Cholesky; diagnostics R(c), kappa(A).

    With a seed the sums hold the re-wrapped residual phases and the returned
    coefficients are c0 + delta.
    """
    A, b = sums["A"], sums["b"]
    nj = len(SOLVED)
    mu = ridge * np.trace(A) / nj
    cf = scipy.linalg.cho_factor(A + mu * np.eye(nj), lower=True)
    cj = scipy.linalg.cho_solve(cf, b)
    resid = (sums["sbb"] - 2.0 * cj @ b + cj @ A @ cj) / sums["sw"]
    c = np.zeros(15)
    c[3:15] = cj
    if seed is not None:
        c[3:15] += np.asarray(seed, dtype=np.float64)[3:15]
    return {"c": c, "residual": float(resid), "kappa": float(np.linalg.cond(A)),
            "sw": sums["sw"], "min_pivot": float(np.min(np.diag(cf[0]).real))}


def estimate_pupil(spectra, k_bf, r, ridge=1e-9, seed=None, bands=PUPIL_BANDS):
    """Eq. 8-10 end to end: sums, then the regularised solve.

    Without a seed the solve runs the coarse-to-fine continuation over
    ``bands`` (fractions of r; an empty tuple gives the paper's single pass).
    The returned diagnostics and sums are those of the last pass over all
    rows; with a seed (given or from the bands) its sums hold the re-wrapped
    phases, so R(c) is the residual of the returned coefficients."""
    if seed is None and bands:
        for f in bands:
            band = aberration_sums(spectra, k_bf, r, seed=seed, k_max=f * r)
            if band["rows"] < MIN_BAND_ROWS:
                continue
            seed = solve_aberration(band, ridge=PUPIL_BAND_RIDGE, seed=seed)["c"]
    sums = aberration_sums(spectra, k_bf, r, seed=seed)
    out = solve_aberration(sums, ridge=ridge, seed=seed)
    out["sums"] = sums
    out["seed"] = None if seed is None else np.asarray(seed, dtype=np.float64).copy()
    return out
