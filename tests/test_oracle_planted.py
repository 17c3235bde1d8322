"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin
catches each one: a flipped sign, a dropped conjugate, a transposed operand."""

import numpy as np
import pytest

import oracle
from oracle import darkfield as odf
from oracle import kk as okk
from oracle import stitch as ost


def _p6_error(n=48, r=9.0):
    from apic_synth.objects import object_smooth
    from oracle.grid import k_grid, circ
    obj = object_smooth(np.random.default_rng(21), n, sigma=1.5)
    c = np.zeros(15)
    c[[3, 4]] = [0.3, -0.2]
    k_bf = np.array([(9, 0), (6, 6), (0, 9), (-6, 6), (-9, 0), (-6, -6), (0, -9), (6, -6)])
    k_j = np.array([11, 3])
    ky, kx = k_grid(n)
    known = np.zeros((n, n), bool)
    for k in k_bf:
        known |= circ(ky + k[1], kx + k[0], r)
    obj_hat = np.fft.fft2(obj)
    img = oracle.forward_images(obj, [k_j], c, r)[0]
    try:
        new_hat, new_known, _ = odf.extend_darkfield(np.where(known, obj_hat, 0), known, img,
                                                     k_j, c, r, ridge=1e-12)
    except np.linalg.LinAlgError:  # a planted mistake may make the gram singular
        return np.inf
    u = new_known & ~known
    return np.abs(new_hat[u] - obj_hat[u]).max() / np.abs(obj_hat[u]).max()


def test_clean_oracle_passes_p6():
    assert _p6_error() < 1e-8


def test_dropped_conjugate_in_c_is_caught(monkeypatch):
    orig = odf.conv_matrix
    monkeypatch.setattr(odf, "conv_matrix", lambda p, q, u, *pad: np.conj(orig(p, q, u, *pad)))
    assert _p6_error() > 1e-3


def test_transposed_difference_in_c_is_caught(monkeypatch):
    def wrong(p_hat, q, u, padded=None):  # P_hat(u - k) instead of P_hat(u + k)
        n = p_hat.shape[0]
        ky = u[:, 0][None, :] - q[:, 0][:, None]
        kx = u[:, 1][None, :] - q[:, 1][:, None]
        return np.conj(odf.gather_signed(p_hat, ky, kx)) / float(n) ** 2
    monkeypatch.setattr(odf, "conv_matrix", wrong)
    assert _p6_error() > 1e-3


def test_flipped_half_plane_is_caught(monkeypatch):
    orig = okk.half_plane_mask
    monkeypatch.setattr(okk, "half_plane_mask", lambda n, k: orig(n, (-k[0], -k[1])))
    from oracle.grid import k_grid
    n, k_i = 64, (12, 5)
    g_hat = np.zeros((n, n), complex)
    g_hat[np.mod(-3, n), np.mod(-4, n)] = 0.3 * n * n
    s = np.exp(np.fft.ifft2(g_hat))
    field, _ = okk.kk_field(np.abs(s) ** 2, k_i)
    assert np.abs(field - s).max() > 1e-2


def test_wrong_correction_sign_is_caught(monkeypatch):
    """Correcting with +phase instead of -phase breaks the stitched spectrum."""
    from oracle.grid import k_grid, circ
    from oracle.zernike import pupil_phase
    n, r = 64, 12.0
    k_bf = np.array([(12, 0), (0, 12), (-12, 0), (0, -12)])
    c = np.zeros(15)
    c[[3, 5]] = [0.2, 0.1]
    obj_hat = np.fft.fft2(np.exp(0.1j * np.random.default_rng(2).standard_normal((n, n))))
    ky, kx = k_grid(n)
    spectra = []
    for k in k_bf:
        sup = circ(ky + k[1], kx + k[0], r)
        ph = pupil_phase(c, ky + k[1], kx + k[0], r) - pupil_phase(c, k[1], k[0], r)
        spectra.append(np.where(sup, obj_hat * np.exp(1j * ph), 0))
    spectra = np.stack(spectra)
    good, known = ost.stitch_brightfield(spectra, k_bf, c, r)
    assert np.abs(good - np.where(known, obj_hat, 0)).max() < 1e-9 * np.abs(obj_hat).max()
    bad, _ = ost.stitch_brightfield(spectra, k_bf, -c, r)
    assert np.abs(bad - np.where(known, obj_hat, 0)).max() > 1e-3 * np.abs(obj_hat).max()
