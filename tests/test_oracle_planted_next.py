"""Plant plausible mistakes in the oracle's pixel-domain pupil solve, patch
assembly, background statistic, colour combination and surrogate fallback
rule (on the CPU), and check that one of their pins catches each."""

import numpy as np
import pytest

import test_oracle_assemble as PA
import test_oracle_background as PB
import test_oracle_fallback as PF
import test_oracle_pixel_pupil as PP
import test_oracle_rgb as PR
from oracle import assemble as oa
from oracle import background as obg
from oracle import fallback as ofb
from oracle import pupil_pixel as opp
from oracle import rgb as orgb


def test_transposed_spectrum_index_in_pixel_rows_is_caught(monkeypatch):
    orig = opp.fft_index
    monkeypatch.setattr(opp, "fft_index", lambda ky, kx, n: orig(kx, ky, n))
    with pytest.raises(AssertionError):
        PP.test_recovers_a_non_zernike_phase()


def test_sign_slip_on_the_led_term_is_caught(monkeypatch):
    """The row operator's last term with the wrong sign: phi(K_l) subtracted
    instead of added."""
    import scipy.sparse as sp
    orig = opp.pixel_system

    def slipped(spectra, k_bf, r):
        D, beta, w, pix = orig(spectra, k_bf, r)
        n = spectra.shape[-1]
        h = n // 2
        _, _, idx = opp.pupil_pixels(n, r)
        k_bf = np.asarray(k_bf, np.int64)
        rows, cols = [], []
        m = 0
        for i, l, ky, kx in opp.pupil_pairs(n, k_bf, r):
            rows.append(np.arange(m, m + len(ky)))
            cols.append(np.full(len(ky), idx[k_bf[l][1] + h, k_bf[l][0] + h]))
            m += len(ky)
        rows, cols = np.concatenate(rows), np.concatenate(cols)
        extra = sp.csr_matrix((np.full(len(rows), -2.0), (rows, cols)), shape=D.shape)
        return (D + extra).tocsr(), beta, w, pix
    monkeypatch.setattr(opp, "pixel_system", slipped)
    monkeypatch.setattr(PP, "pixel_system", slipped)
    with pytest.raises(AssertionError):
        PP.test_null_space_is_piston_tip_tilt(64, 8)
    with pytest.raises(AssertionError):
        PP.test_recovers_a_non_zernike_phase()


def test_conjugated_overlap_correlation_is_caught(monkeypatch):
    orig = oa.overlap_matrix
    monkeypatch.setattr(oa, "overlap_matrix", lambda f, p, min_overlap=1: np.conj(orig(f, p, min_overlap)))
    with pytest.raises(AssertionError):
        PA.test_cut_tiles_reassemble_exactly(4.0)


def test_half_pixel_ramp_slip_is_caught(monkeypatch):
    def slipped(n, width):
        v = np.arange(n).astype(float)
        return np.minimum(1.0, np.minimum((v + 1e-9) / width, (n - v) / width))
    monkeypatch.setattr(oa, "ramp", slipped)
    with pytest.raises(AssertionError):
        PA.test_ramp_closed_form()


def test_sample_variance_divisor_is_caught(monkeypatch):
    def sample(img):
        x = np.asarray(img, np.float64)
        return float(np.var(x, ddof=1) / x.mean() ** 2)
    monkeypatch.setattr(obg, "relative_variance", sample)
    with pytest.raises(AssertionError):
        PB.test_cosine_closed_form(8, 1, 0, 0.3)


def test_inverted_grey_world_gains_are_caught(monkeypatch):
    def inverted(fields_rgb):
        m = np.array([np.mean(np.abs(f)) for f in fields_rgb])
        return m / m.mean()
    monkeypatch.setattr(orgb, "grey_world_gains", inverted)
    with pytest.raises(AssertionError):
        PR.test_constant_channels_come_out_grey()


def test_sign_slip_in_the_expanded_residual_is_caught(monkeypatch):
    """S_bb + 2 c.b + c.A c instead of S_bb - 2 c.b + c.A c."""
    def slipped(sums, c12):
        c = np.asarray(c12, np.float64)
        return float((sums["sbb"] + 2.0 * (c @ sums["b"]) + c @ sums["A"] @ c) / sums["sw"])
    monkeypatch.setattr(ofb, "residual", slipped)
    with pytest.raises(AssertionError):
        PF.test_residual_matches_brute_force_over_rows()


def test_inverted_rho_threshold_is_caught(monkeypatch):
    """Closed form kept when the surrogate is within rho_max instead of beyond."""
    def inverted(sums, c_cf, c_sur, kappa, rho_max, kappa_max, resid_max):
        r_cf = ofb.residual(sums, c_cf)
        rho = float(np.sqrt(max(0.0, ofb.residual(sums, c_sur) - r_cf)))
        keep_cf = rho <= rho_max and kappa <= kappa_max and r_cf <= resid_max
        return (not keep_cf), rho, r_cf
    monkeypatch.setattr(ofb, "choose", inverted)
    with pytest.raises(AssertionError):
        PF.test_decision_at_the_thresholds()
