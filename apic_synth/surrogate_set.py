"""Synthetic tiles for the learned pupil surrogate (128 x 128, 16 NA-matched
images on the NA 0.25 ring, no darkfield), generated on the target device with
torch.

* Field model: c_4..c_15 quadratic in the normalised position (u, v) with the
  coefficients of ``field_model_quadratic`` (default_rng([2407, 20469])), scaled so
  that max |c| over a 64 x 64 grid of [-1, 1]^2 equals ``max_abs``.
* Content tiles: amplitude 0.85..1 and phase 0..pi, periodic Gaussian
  smoothing sigma = 2 px (the smooth-object recipe).  Background tiles: amplitude
  1 - a_bg (1 - minmax(noise)) and smooth phase with standard deviation drawn
  from U(bg_lo, bg_hi) rad, the amplitude texture a_bg scaled with the same
  draw (0.01 at 0.02 rad), so the lowest draws approach blank glass.
* Poisson noise at ``photons`` per unit intensity.  All draws come from one
  torch generator seeded with ``seed``; results depend on the device type.
"""

import math

import numpy as np
import torch

from .configs import field_model_quadratic
from .imaging import form_images
from .leds import led_ring

N = 128
N_BF = 16


def geometry(n=N, n_bf=N_BF):
    k_bf = np.array(led_ring(n, 0.25, n_bf, 0.0, True))
    return {"n": n, "dx_um": 0.4, "wavelength_um": 0.52, "na_obj": 0.25, "k_bf": k_bf,
            "k_df": np.zeros((0, 2), np.int64), "upsample": 1}


def field_coeffs(max_abs=0.3):
    """Scaled quadratic field model: (12, 6) coefficients of (1, u, v, u^2, uv, v^2)."""
    g = (np.arange(64) - 31.5) / 31.5
    gu, gv = np.meshgrid(g, g)
    _, a = field_model_quadratic(gu.ravel(), gv.ravel(), max_abs=max_abs)
    return a


def pupil_at(a, uv):
    """True Noll coefficients (T, 15) at positions uv (T, 2)."""
    u, v = uv[:, 0], uv[:, 1]
    basis = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], axis=-1)
    c = np.zeros((len(uv), 15))
    c[:, 3:15] = basis @ a.T
    return c


def _smooth(x, sigma):
    n = x.shape[-1]
    f = torch.fft.fftfreq(n, device=x.device, dtype=x.dtype)
    h = torch.exp(-2.0 * math.pi ** 2 * sigma ** 2 * (f[:, None] ** 2 + f[None, :] ** 2))
    return torch.fft.ifft2(torch.fft.fft2(x) * h).real


def _minmax(x):
    lo = x.amin(dim=(-2, -1), keepdim=True)
    hi = x.amax(dim=(-2, -1), keepdim=True)
    return (x - lo) / (hi - lo)


def make_tiles(uv, background, seed, device, max_abs=0.3, photons=1e4, chunk=256, bg_lo=0.005,
               bg_hi=0.02, n=N):
    """float32 images (T, 16, n, n) on device (default n = 128) and true
    coefficients (T, 15)."""
    geom = geometry(n)
    r = geom["na_obj"] * geom["n"] * geom["dx_um"] / geom["wavelength_um"]
    a = field_coeffs(max_abs)
    c_true = pupil_at(a, np.asarray(uv, np.float64))
    T = len(uv)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = torch.empty((T, N_BF, n, n), dtype=torch.float32, device=device)
    bg = torch.as_tensor(np.asarray(background, bool), device=device)
    for s in range(0, T, chunk):
        e = min(T, s + chunk)
        m = e - s
        u0 = torch.rand((m, n, n), generator=gen, device=device, dtype=torch.float64)
        g0 = torch.randn((m, n, n), generator=gen, device=device, dtype=torch.float64)
        lvl = bg_lo + (bg_hi - bg_lo) * torch.rand((m, 1, 1), generator=gen, device=device,
                                                   dtype=torch.float64)
        sm_u, sm_g = _smooth(u0, 2.0), _smooth(g0, 2.0)
        b = bg[s:e, None, None]
        amp_bg = 1.0 - (0.5 * lvl) * (1.0 - _minmax(sm_u))
        amp = torch.where(b, amp_bg, 0.85 + 0.15 * _minmax(sm_u))
        psi_bg = sm_g / sm_g.std(dim=(-2, -1), keepdim=True) * lvl
        psi = torch.where(b, psi_bg, math.pi * _minmax(sm_g))
        obj = amp * torch.exp(1j * psi)
        imgs = form_images(obj, c_true[s:e], [tuple(k) for k in geom["k_bf"]], r, device=device,
                           dtype=torch.float64)
        lam = (imgs * photons).clamp_min(0.0)
        out[s:e] = (torch.poisson(lam, generator=gen) / photons).to(torch.float32)
    return out, c_true
