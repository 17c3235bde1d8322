"""The darkfield chain transforms |P|^2 and the darkfield image I_j together,
as the real and imaginary parts of one complex FFT (Eq. 13 needs both
spectra). These CPU checks pin the separation with the component formulas the
right-hand-side pass and the gram's Toeplitz term use, against two separate
FFTs, on the grid index conventions of the kernels (-k at ((N - y) mod N,
(N - x) mod N))."""

import numpy as np
import pytest


def _neg(a):
    """a(-k) on an FFT-ordered N x N grid."""
    return np.roll(a[::-1, ::-1], 1, axis=(0, 1))


def _separate_rhs(z):
    """conj(fft2(I) - fft2(|P|^2)) from z(k) and z(-k), component by component
    as the right-hand-side pass computes it."""
    z1, z2 = z, _neg(z)
    re = 0.5 * ((z1.imag + z2.imag) - (z1.real + z2.real))
    im = 0.5 * ((z1.real - z2.real) + (z1.imag - z2.imag))
    return re + 1j * im


def _separate_toeplitz(z):
    """fft2(|P|^2) from z(d) and z(-d), as the gram's epilogue computes it."""
    z1, z2 = z, _neg(z)
    return 0.5 * (z1.real + z2.real) + 0.5j * (z1.imag - z2.imag)


@pytest.mark.parametrize("n", [8, 64, 256])
def test_one_complex_fft_carries_both_real_spectra(n):
    rng = np.random.default_rng(n)
    p = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    pp = np.abs(p) ** 2
    img = rng.poisson(1e4 * (0.5 + rng.random((n, n)))).astype(np.float64)
    z = np.fft.fft2(pp + 1j * img)
    f_pp, f_img = np.fft.fft2(pp), np.fft.fft2(img)
    scale = np.abs(z).max()
    assert np.abs(_separate_toeplitz(z) - f_pp).max() < 1e-13 * scale
    assert np.abs(_separate_rhs(z) - np.conj(f_img - f_pp)).max() < 1e-13 * scale


def test_neg_index_matches_the_kernel_mirror():
    n = 16
    a = np.arange(n * n).reshape(n, n)
    m = _neg(a)
    for y in range(n):
        for x in range(n):
            assert m[y, x] == a[(n - y) & (n - 1), (n - x) & (n - 1)]


def test_a_sign_slip_in_the_separation_is_caught():
    """Planted mistake: swapping the roles of z(k) and z(-k) in the imaginary
    part of the Toeplitz term conjugates fft2(|P|^2) and fails the check."""
    n = 32
    rng = np.random.default_rng(3)
    pp = rng.random((n, n))
    img = rng.random((n, n))
    z = np.fft.fft2(pp + 1j * img)
    wrong = 0.5 * (z.real + _neg(z).real) + 0.5j * (_neg(z).imag - z.imag)
    assert np.abs(wrong - np.fft.fft2(pp)).max() > 1e-3
