"""Pins of the oracle's pixel-domain pupil solve (Eq. 10 with one unknown per
pupil pixel).

* The null space of D is exactly piston, tip and tilt (a wrong sign on the
  phi(K_i) / phi(K_l) terms or a swapped shift adds or removes directions),
  except for LED layouts on a parity sublattice, where the checkerboard
  joins it and the minimum-norm solution carries none of it.
* A phase that no Zernike expansion of order 4 holds is recovered exactly,
  up to that null space, from spectra built by Eq. 9's structure.
* For a phase in the span of Z_4..Z_15 the pixel solve's Zernike summary and
  the Zernike-basis solve both return the true coefficients.
"""

import numpy as np
import pytest

from apic_synth.leds import led_rings
from apic_synth.objects import object_smooth
from oracle.aberration import estimate_pupil
from oracle.grid import circ, fft_index, k_grid
from oracle.pupil_pixel import pixel_system, pupil_pixels, solve_pixel_pupil
from oracle.zernike import zernike


def _geometry(n=64, count=8):
    r = 0.25 * n * 0.4 / 0.52
    return n, r, np.asarray(led_rings(n, [(0.25, count, 0.0, True)]), np.int64)


def _spectra(n, r, k_bf, phi_of, seed=0):
    """Eq. 9 structure: s_i(k) = O(k) exp(j [phi(k + k_i) - phi(k_i)]) on
    Circ(k + k_i), for a smooth random object spectrum O."""
    obj = object_smooth(np.random.default_rng([seed, 0, 0]), n)
    O = np.fft.fft2(obj)
    ky, kx = k_grid(n)
    out = np.zeros((len(k_bf), n, n), complex)
    for i, (kxi, kyi) in enumerate(k_bf):
        sup = circ(ky + kyi, kx + kxi, r)
        ph = phi_of(ky + kyi, kx + kxi) - phi_of(np.array(kyi), np.array(kxi))
        out[i] = np.where(sup, O * np.exp(1j * ph), 0.0)
    return out


def _gauge_free(phi, ky, kx):
    """phi minus its least-squares fit by 1, kx, ky over the pupil pixels."""
    B = np.stack([np.ones_like(kx, dtype=float), kx, ky], axis=1).astype(float)
    coef, *_ = np.linalg.lstsq(B, phi, rcond=None)
    return phi - B @ coef


@pytest.mark.parametrize("n,count", [(64, 8), (128, 16)])
def test_null_space_is_piston_tip_tilt(n, count):
    n, r, k_bf = _geometry(n, count)
    spectra = _spectra(n, r, k_bf, lambda y, x: 0.0 * x)
    D, beta, w, (ky, kx) = pixel_system(spectra, k_bf, r)
    for v in (np.ones(len(kx)), kx.astype(float), ky.astype(float)):
        assert np.abs(D @ v).max() < 1e-12
    ev = np.linalg.eigvalsh((D.T @ D).toarray())
    assert np.sum(ev < 1e-9 * ev.max()) == 3
    assert ev[3] > 1e-6 * ev.max()


def test_lattice_mode_joins_the_null_space():
    """128 px, 8 LEDs: every LED has kx + ky even, so (-1)^(kx + ky) cancels in
    every row; the minimum-norm solution carries none of it."""
    n, r, k_bf = _geometry(128, 8)
    assert np.all((k_bf.sum(axis=1) % 2) == 0)
    rng = np.random.default_rng(7)
    c = np.zeros(15)
    c[3:8] = rng.uniform(-0.2, 0.2, 5)
    spectra = _spectra(n, r, k_bf, lambda y, x: sum(c[j - 1] * zernike(j, np.asarray(y),
                                                                       np.asarray(x), r)
                                                     for j in range(4, 9)), seed=4)
    D, beta, w, (ky, kx) = pixel_system(spectra, k_bf, r)
    checker = (-1.0) ** (kx + ky)
    assert np.abs(D @ checker).max() < 1e-12
    out = solve_pixel_pupil(spectra, k_bf, r)
    assert out["null_dim"] == 4
    assert abs(out["phi"] @ checker) < 1e-9 * np.linalg.norm(out["phi"]) * np.sqrt(len(kx))


def test_recovers_a_non_zernike_phase():
    n, r, k_bf = _geometry()
    rng = np.random.default_rng(3)
    centres = rng.uniform(-0.7 * r, 0.7 * r, (5, 2))
    amps = rng.uniform(-0.4, 0.4, 5)

    def phi_of(y, x):
        y = np.asarray(y, float)
        x = np.asarray(x, float)
        return sum(a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (0.15 * r) ** 2)
                   for a, (cx, cy) in zip(amps, centres))

    spectra = _spectra(n, r, k_bf, phi_of, seed=1)
    out = solve_pixel_pupil(spectra, k_bf, r)
    assert out["null_dim"] == 3
    ky, kx = out["ky"], out["kx"]
    truth = _gauge_free(phi_of(ky, kx), ky, kx)
    assert np.abs(out["phi"] - truth).max() < 1e-9
    # the bumps are not in the span of Z_1..Z_15: the summary misses part of them
    Z = np.stack([zernike(j, ky, kx, r) for j in range(1, 16)], axis=1)
    fit = Z @ np.linalg.lstsq(Z, truth, rcond=None)[0]
    assert np.linalg.norm(truth - fit) > 0.1 * np.linalg.norm(truth)
    # the map holds phi at the pixels in FFT order and 0 elsewhere
    yy, xx = fft_index(ky, kx, n)
    assert np.array_equal(out["phi_map"][yy, xx], out["phi"])
    assert np.count_nonzero(out["phi_map"]) <= len(ky)


def test_zernike_phase_matches_zernike_basis_solve():
    n, r, k_bf = _geometry(n=128, count=16)
    c_true = np.zeros(15)
    c_true[[3, 4, 5, 6, 7, 10, 13]] = [0.3, -0.2, 0.15, 0.1, -0.12, 0.08, 0.05]

    def phi_of(y, x):
        return sum(c_true[j - 1] * zernike(j, np.asarray(y), np.asarray(x), r) for j in range(4, 16))

    spectra = _spectra(n, r, k_bf, phi_of, seed=2)
    pix = solve_pixel_pupil(spectra, k_bf, r)
    zb = estimate_pupil(spectra, k_bf, r, ridge=1e-14)
    assert np.abs(pix["c"] - c_true).max() < 1e-8
    assert np.abs(zb["c"] - c_true).max() < 1e-8
    assert np.all(pix["c"][:3] == 0)


@pytest.mark.parametrize("n,count", [(64, 8), (128, 8), (128, 16)])
def test_lsqr_route_equals_eigendecomposition_route(n, count):
    """The LSQR route (for pupils too large for a dense normal matrix) reaches
    the same minimum-norm solution as the eigendecomposition on the range,
    also where the checkerboard joins the null space (128 px / 8 LEDs), on
    noisy spectra whose rows are inconsistent."""
    n, r, k_bf = _geometry(n, count)
    rng = np.random.default_rng([n, count, 7])
    s = _spectra(n, r, k_bf, lambda ky, kx: 0.3 * np.sin(0.2 * kx) + 0.01 * ky * ky / r)
    s = s * np.exp(1j * rng.normal(0, 0.05, s.shape)) * (s != 0)
    a = solve_pixel_pupil(s, k_bf, r)
    b = solve_pixel_pupil(s, k_bf, r, method="lsqr")
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-7
    assert np.abs(a["c"] - b["c"]).max() < 1e-9
