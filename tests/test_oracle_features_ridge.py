"""Pins of two oracle parts that the parity tests run but earlier pins left
open: the surrogate's spectral-overlap features (the weight sums of Eq. 10's
rows per cell) and the darkfield solve at its default ridge (Eq. 13 as
Tikhonov least squares), plus the correlation routes of the T - E gram.

The features are checked by a conservation law (every row's weight lands in
exactly one cell), by hand-placed pairs and frequencies at and beside the bin
edges, and by a brute-force count over every row with an independent
formulation of the bins; planted mistakes (a band edge at r instead of 2r, an
angle bin shifted by one) fail these.  The darkfield solve is checked against
the Tikhonov solution written through the singular value decomposition of C
(no normal equations), with C built by an explicit double loop.
"""

import numpy as np
import pytest

from oracle import aberration as oab
from oracle import darkfield as odf
from oracle.grid import k_grid, circ, fft_index
from oracle.zernike import pupil_phase
from apic_synth.objects import object_smooth
import oracle


# ------------------------------------------------------------ surrogate features
def _random_spectra(n, n_img, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_img, n, n)) + 1j * rng.standard_normal((n_img, n, n))


@pytest.mark.parametrize("n,r,k_bf", [
    (64, 12.3, [(12, 0), (9, 8), (0, 12), (-8, 9), (-12, 0), (-9, -8), (0, -12), (8, -9)]),
    (48, 9.0, [(9, 0), (0, 9), (-9, 0), (0, -9), (6, 6), (-6, 6)]),
])
def test_feature_weights_are_conserved(n, r, k_bf):
    """sum over the 32 cells of expm1(feature) * N^4 equals the total weight
    sum of Eq. 10's rows: no row is lost or counted twice."""
    s = oab.aberration_sums(_random_spectra(n, len(k_bf), n), k_bf, r)
    total = np.sum(np.expm1(s["features"])) * float(n) ** 4
    assert abs(total - s["sw"]) < 1e-10 * s["sw"]
    # with unit-modulus spectra every row weighs 1: the cell sums count rows
    ones = np.exp(1j * np.angle(_random_spectra(n, len(k_bf), n + 1)))
    s1 = oab.aberration_sums(ones, k_bf, r)
    counts = np.expm1(s1["features"]) * float(n) ** 4
    assert np.allclose(counts, np.round(counts), atol=1e-6)
    assert int(round(counts.sum())) == s1["rows"]


# (k_i, k_l, K as (ky, kx), expected cell) with r = 20: the bands of |K|/(2r)
# have edges at |K| = 10, 20, 30, 40 and the angle bins at multiples of pi/8;
# a value on an edge belongs to the lower bin.
R_HAND = 20.0
HAND = [
    ((1, 0), (1, 1), (0, 10), 1 * 4 + 0),    # pi/4 on an edge; |K| = 10 on an edge
    ((1, 0), (1, 1), (0, 11), 1 * 4 + 1),
    ((1, 0), (0, 1), (6, 8), 3 * 4 + 0),     # pi/2 on an edge; |K| = 10 on an edge
    ((1, 0), (0, 1), (12, 16), 3 * 4 + 1),   # |K| = 20 on an edge
    ((1, 0), (0, 1), (0, 21), 3 * 4 + 2),
    ((1, 0), (-1, 1), (18, 24), 5 * 4 + 2),  # 3 pi/4; |K| = 30
    ((1, 0), (-1, 0), (0, 31), 7 * 4 + 3),   # pi
    ((1, 0), (-1, 0), (24, 32), 7 * 4 + 3),  # |K| = 40 = 2r
    ((1, 0), (2, 1), (0, 1), 1 * 4 + 0),     # atan(1/2) = 1.18 pi/8
    ((1, 0), (5, 1), (1, 1), 0 * 4 + 0),     # 0.50 pi/8
    ((1, 0), (1, 2), (-7, -7), 2 * 4 + 0),   # 2.82 pi/8; |K| = 9.9
    ((3, 4), (4, 3), (-30, 0), 0 * 4 + 2),   # 0.72 pi/8
    ((-3, 4), (4, -3), (0, -25), 7 * 4 + 2),  # 7.28 pi/8
    ((0, 7), (-7, 7), (5, 0), 1 * 4 + 0),    # pi/4 between rotated vectors
]


def _hand_mismatches(cell_fn):
    bad = 0
    for k_i, k_l, K, want in HAND:
        got = cell_fn(np.array(k_i), np.array(k_l), np.array([K[0]]), np.array([K[1]]), R_HAND)
        bad += int(np.asarray(got).reshape(-1)[0] != want)
    return bad


def test_feature_cells_hand_placed():
    assert _hand_mismatches(oab.feature_cell) == 0


def _brute_counts(n, r, k_bf):
    """Row counts per cell by enumerating every pair and every K of its
    overlap, with the bins formulated independently: the angle from atan2 of
    the cross and dot products, and both bin indices as the number of edges
    strictly passed (beyond a 1e-9 guard)."""
    counts = np.zeros(32, dtype=np.int64)
    half = n // 2
    for i in range(len(k_bf)):
        for l in range(i + 1, len(k_bf)):
            (ax, ay), (bx, by) = k_bf[i], k_bf[l]
            ang = np.arctan2(abs(ax * by - ay * bx), ax * bx + ay * by)
            abin = sum(ang > m * np.pi / 8 + 1e-9 for m in range(1, 8))
            for Ky in range(-half, half):
                for Kx in range(-half, half):
                    if Ky == 0 and Kx == 0:
                        continue
                    if (Kx + ax) ** 2 + (Ky + ay) ** 2 > r * r:
                        continue
                    if (Kx + bx) ** 2 + (Ky + by) ** 2 > r * r:
                        continue
                    rho = np.hypot(Kx, Ky) / (2 * r)
                    band = sum(rho > m / 4 + 1e-9 for m in range(1, 4))
                    counts[abin * 4 + band] += 1
    return counts


def _oracle_counts(n, r, k_bf):
    ones = np.ones((len(k_bf), n, n), dtype=np.complex128)
    s = oab.aberration_sums(ones, k_bf, r)
    return np.round(np.expm1(s["features"]) * float(n) ** 4).astype(np.int64)


BRUTE_CASE = (32, 6.0, [(6, 0), (4, 4), (0, 6), (-4, 4), (-6, 0), (-4, -4), (0, -6), (4, -4)])


def test_feature_cells_brute_force():
    n, r, k_bf = BRUTE_CASE
    want = _brute_counts(n, r, k_bf)
    assert want.sum() > 0 and np.count_nonzero(want) >= 8
    assert np.array_equal(_oracle_counts(n, r, k_bf), want)


def _cell_band_edge_at_r(k_i, k_l, K_y, K_x, r):
    ki, kl = np.asarray(k_i, float), np.asarray(k_l, float)
    ang = np.arccos(np.clip(ki @ kl / (np.linalg.norm(ki) * np.linalg.norm(kl)), -1, 1))
    abin = int(np.clip(np.ceil(ang / (np.pi / 8) - 1e-9) - 1, 0, 7))
    rho = np.hypot(K_x, K_y) / r                      # planted: |K| / r
    band = np.clip(np.ceil(4 * rho - 1e-9) - 1, 0, 3).astype(np.int64)
    return abin * 4 + band


def _cell_angle_shifted(k_i, k_l, K_y, K_x, r):
    ki, kl = np.asarray(k_i, float), np.asarray(k_l, float)
    ang = np.arccos(np.clip(ki @ kl / (np.linalg.norm(ki) * np.linalg.norm(kl)), -1, 1))
    abin = int(np.clip(np.floor(ang / (np.pi / 8)), 0, 7))   # planted: edges go up
    rho = np.hypot(K_x, K_y) / (2 * r)
    band = np.clip(np.ceil(4 * rho - 1e-9) - 1, 0, 3).astype(np.int64)
    return abin * 4 + band


_CLEAN_CELL = oab.feature_cell


def _cell_angle_off_by_one(k_i, k_l, K_y, K_x, r):
    return np.minimum(_CLEAN_CELL(k_i, k_l, K_y, K_x, r) + 4, 31)   # planted: next angle bin


@pytest.mark.parametrize("planted", [_cell_band_edge_at_r, _cell_angle_shifted,
                                     _cell_angle_off_by_one])
def test_planted_feature_mistakes_are_caught(monkeypatch, planted):
    assert _hand_mismatches(planted) > 0
    monkeypatch.setattr(oab, "feature_cell", planted)
    n, r, k_bf = BRUTE_CASE
    assert not np.array_equal(_oracle_counts(n, r, k_bf), _brute_counts(n, r, k_bf))


# ------------------------------------------------------------ darkfield ridge
def _small_darkfield(n=40, r=7.5, seed=31):
    rng = np.random.default_rng(seed)
    obj = object_smooth(rng, n, sigma=1.5)
    c = np.zeros(15)
    c[[3, 4, 6]] = [0.3, -0.2, 0.15]
    k_bf = np.array([(7, 0), (5, 5), (0, 7), (-5, 5), (-7, 0), (-5, -5), (0, -7), (5, -5)])
    k_j = np.array([9, 3])
    ky, kx = k_grid(n)
    known = np.zeros((n, n), bool)
    for k in k_bf:
        known |= circ(ky + k[1], kx + k[0], r)
    obj_hat = np.fft.fft2(obj)
    img = oracle.forward_images(obj, [k_j], c, r)[0]
    # a Poisson-like perturbation so that the system is not exactly consistent
    img = img + 1e-3 * rng.standard_normal(img.shape) * np.sqrt(np.maximum(img, 0))
    return obj_hat, known, img, k_j, c, r


def _c_by_loops(p_hat, q, u):
    n = p_hat.shape[0]
    cm = np.zeros((len(q), len(u)), dtype=np.complex128)
    for a in range(len(q)):
        for b in range(len(u)):
            yy, xx = q[a, 0] + u[b, 0], q[a, 1] + u[b, 1]
            if -n // 2 <= yy < n // 2 and -n // 2 <= xx < n // 2:
                cm[a, b] = np.conj(p_hat[yy % n, xx % n]) / n ** 2
    return cm


def _svd_pin_error(gram, ridge_used):
    """Max deviation of the oracle's solve (run with ``ridge_used``) from the
    Tikhonov solution at lambda = 1e-4, x = V diag(s / (s^2 + lam')) U^H b
    with lam' = lambda ||C||_F^2 / N_u, computed from the SVD of C (built by
    loops), never forming C^H C.  Also returns the distance of that solution
    from the unregularised least-squares one, relative to |x|."""
    obj_hat, known, img, k_j, c, r = _small_darkfield()
    n = obj_hat.shape[0]
    start = np.where(known, obj_hat, 0)
    _, _, info = odf.extend_darkfield(start, known, img, k_j, c, r, gram=gram, ridge=ridge_used)
    sets = odf.darkfield_sets(n, k_j, known, r)
    ky, kx = k_grid(n)
    p_hat = np.where(sets["P_mask"], start * np.exp(1j * pupil_phase(c, ky + k_j[1], kx + k_j[0], r)), 0)
    cm = _c_by_loops(p_hat, sets["Q"], sets["U"])
    f_img = np.fft.fft2(img)
    f_pp = np.fft.fft2(np.abs(np.fft.ifft2(p_hat)) ** 2)
    yy, xx = fft_index(sets["Q"][:, 0], sets["Q"][:, 1], n)
    b = np.conj(f_img[yy, xx] - f_pp[yy, xx])
    uu, s, vh = np.linalg.svd(cm, full_matrices=False)
    lam = 1e-4 * np.sum(np.abs(cm) ** 2) / len(sets["U"])
    x = vh.conj().T @ ((s / (s * s + lam)) * (uu.conj().T @ b))
    x0 = np.linalg.lstsq(cm, b, rcond=None)[0]
    scale = np.abs(x).max()
    return np.abs(info["x"] - x).max() / scale, np.abs(x0 - x).max() / scale, info["n_u"]


@pytest.mark.parametrize("gram", ["fullq", "t-e"])
def test_darkfield_default_ridge_equals_svd_tikhonov(gram):
    err, ridge_effect, _ = _svd_pin_error(gram, 1e-4)
    assert err < 1e-9
    # the ridge is not negligible on this system: dropping it moves x clearly
    assert ridge_effect > 1e-6


@pytest.mark.parametrize("scale", ["times_nu", "over_nu"])
def test_planted_ridge_scale_is_caught(scale):
    """A ridge of lambda tr(G) (not divided by N_u) or lambda tr(G) / N_u^2
    fails the SVD pin."""
    _, _, nu = _svd_pin_error("fullq", 1e-4)
    wrong = 1e-4 * nu if scale == "times_nu" else 1e-4 / nu
    err, _, _ = _svd_pin_error("fullq", wrong)
    assert err > 1e-7


# ------------------------------------------------------------ T - E correlations
def test_autocorrelation_grid_matches_direct_sum():
    obj_hat, known, img, k_j, c, r = _small_darkfield(n=32, r=6.0, seed=5)
    n = obj_hat.shape[0]
    sets = odf.darkfield_sets(n, k_j, known, r)
    rng = np.random.default_rng(3)
    p_hat = np.zeros((n, n), complex)
    pm = sets["P_mask"]
    p_hat[pm] = rng.normal(size=pm.sum()) + 1j * rng.normal(size=pm.sum())
    rg = odf.autocorrelation_grid(p_hat)
    d = np.array([(0, 0), (1, 0), (0, -3), (5, 7), (-9, 4), (12, -12), (15, 15), (-16, 0)])
    direct = odf.autocorrelation(p_hat, sets["P"], d)
    got = rg[np.mod(d[:, 0], 2 * n), np.mod(d[:, 1], 2 * n)]
    assert np.abs(got - direct).max() < 1e-12 * np.abs(direct).max()


def test_rhs_by_correlation_matches_loops():
    obj_hat, known, img, k_j, c, r = _small_darkfield(n=32, r=6.0, seed=6)
    n = obj_hat.shape[0]
    sets = odf.darkfield_sets(n, k_j, known, r)
    rng = np.random.default_rng(4)
    p_hat = np.zeros((n, n), complex)
    pm = sets["P_mask"]
    p_hat[pm] = rng.normal(size=pm.sum()) + 1j * rng.normal(size=pm.sum())
    q, u = sets["Q"], sets["U"]
    b = rng.normal(size=len(q)) + 1j * rng.normal(size=len(q))
    want = _c_by_loops(p_hat, q, u).conj().T @ b
    got = odf.rhs_by_correlation(p_hat, q, u, b)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_t_minus_e_path_equals_full_q_path():
    obj_hat, known, img, k_j, c, r = _small_darkfield(n=48, r=9.0, seed=8)
    start = np.where(known, obj_hat, 0)
    a, _, ia = odf.extend_darkfield(start, known, img, k_j, c, r, gram="fullq")
    b, _, ib = odf.extend_darkfield(start, known, img, k_j, c, r, gram="t-e")
    assert np.abs(ia["gram"] - ib["gram"]).max() < 1e-12 * np.abs(ia["gram"]).max()
    assert np.abs(ia["rhs"] - ib["rhs"]).max() < 1e-12 * np.abs(ia["rhs"]).max()
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()
