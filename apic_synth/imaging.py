"""Batched image formation with torch (Eq. 1-2 in the shifted frame of Eq. 3),
for synthesising many tiles on the GPU or CPU.  This is the microscope's side
of the problem, not a reconstruction step.

For each tile t and illumination k_i:
    S'_i(k) = O_hat_t(k) Circ(k + k_i) exp(j phi_t(k + k_i)),  I = |ifft2 S'_i|^2
with phi_t the tile's pupil phase from Noll coefficients, evaluated here from
the closed-form radial polynomials of orders n <= 4.
"""

import math

import numpy as np
import torch

# (n, m) of Noll j = 1..15 and the closed-form radial polynomials R_n^|m|.
_NOLL = [(0, 0), (1, 1), (1, -1), (2, 0), (2, -2), (2, 2), (3, -1), (3, 1), (3, -3), (3, 3),
         (4, 0), (4, 2), (4, -2), (4, 4), (4, -4)]
_RADIAL = {
    (0, 0): lambda p: torch.ones_like(p),
    (1, 1): lambda p: p,
    (2, 0): lambda p: 2 * p ** 2 - 1,
    (2, 2): lambda p: p ** 2,
    (3, 1): lambda p: 3 * p ** 3 - 2 * p,
    (3, 3): lambda p: p ** 3,
    (4, 0): lambda p: 6 * p ** 4 - 6 * p ** 2 + 1,
    (4, 2): lambda p: 4 * p ** 4 - 3 * p ** 2,
    (4, 4): lambda p: p ** 4,
}


def _basis(qy, qx, r):
    """(15, ...) orthonormal Zernike values at integer frequencies (qy, qx)."""
    rho = torch.sqrt(qx * qx + qy * qy) / r
    th = torch.atan2(qy, qx)
    out = []
    for n, m in _NOLL:
        rad = _RADIAL[(n, abs(m))](rho)
        if m == 0:
            out.append(math.sqrt(n + 1) * rad)
        elif m > 0:
            out.append(math.sqrt(2 * (n + 1)) * rad * torch.cos(m * th))
        else:
            out.append(math.sqrt(2 * (n + 1)) * rad * torch.sin(-m * th))
    return torch.stack(out)


def form_images(objects, coeffs, k_list, r, device="cpu", dtype=torch.float64):
    """Noise-free intensities for a batch of tiles.

    objects  complex array-like (T, N, N)
    coeffs   (T, 15) Noll coefficients of each tile's true pupil
    k_list   (n, 2) integer (kx, ky)
    Returns a torch tensor (T, n, N, N) of ``dtype`` on ``device``.
    """
    cdtype = torch.complex128 if dtype == torch.float64 else torch.complex64
    if isinstance(objects, torch.Tensor):
        obj = objects.to(device=device, dtype=cdtype)
    else:
        obj = torch.as_tensor(np.asarray(objects), device=device).to(cdtype)
    c = torch.as_tensor(np.asarray(coeffs, dtype=np.float64), device=device).to(dtype)
    t_count, n, _ = obj.shape
    f = torch.fft.fftfreq(n, device=device, dtype=dtype) * n
    ky = f[:, None].expand(n, n)
    kx = f[None, :].expand(n, n)
    obj_hat = torch.fft.fft2(obj)
    out = torch.empty((t_count, len(k_list), n, n), dtype=dtype, device=device)
    for idx, (kix, kiy) in enumerate(k_list):
        qy = ky + float(kiy)
        qx = kx + float(kix)
        support = (qx * qx + qy * qy) <= r * r
        basis = _basis(qy, qx, r)                                # (15, N, N)
        phase = torch.einsum("tj,jyx->tyx", c, basis)            # (T, N, N)
        spec = torch.where(support, obj_hat * torch.exp(1j * phase.to(cdtype)),
                           torch.zeros((), dtype=cdtype, device=device))
        out[:, idx] = torch.fft.ifft2(spec).abs() ** 2
    return out


def add_poisson(images, photons, seed, device="cpu"):
    """Shot noise: I <- Poisson(photons * I) / photons (float64 draw)."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    lam = (images.to(torch.float64) * photons).clamp_min(0.0)
    return torch.poisson(lam, generator=gen) / photons
