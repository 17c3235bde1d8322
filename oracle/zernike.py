"""Zernike basis for the pupil phase (not in the paper; the paper solves Eq. 10
for the pupil phase on the pixel grid).  The unknown here is the vector of Noll
coefficients c_4..c_15 (Noll 1976, J. Opt. Soc. Am. 66, 207):

* Noll index j -> (n, m); even j carries cos(m theta), odd j sin(|m| theta);
* R_n^|m|(rho) from the factorial sum;
* normalisation sqrt(n+1) for m = 0, sqrt(2(n+1)) otherwise, so that
  (1/pi) * integral over the unit disk of Z_j Z_j' = delta_jj';
* rho = |k| / r and theta = atan2(ky, kx), ky being the row (y) frequency.

Piston, tip and tilt (j = 1..3) lie in the null space of Eq. 10's operator
(a constant or linear phase cancels in phi(K+K_i) - phi(K+K_l) - phi(K_i) +
phi(K_l)), so the solve fixes them to zero.
"""

from math import factorial

import numpy as np

N_ZERNIKE = 15
SOLVED = tuple(range(4, 16))  # Noll indices carried by the aberration solve


def noll_nm(j):
    """Radial order n and signed azimuthal order m of Noll index j >= 1."""
    if j < 1:
        raise ValueError("Noll index starts at 1")
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    pos = j - n * (n + 1) // 2 - 1
    orders = []
    for am in range(n % 2, n + 1, 2):
        orders += [0] if am == 0 else [am, am]
    am = orders[pos]
    if am == 0:
        return n, 0
    return n, (am if j % 2 == 0 else -am)


def radial(n, am, rho):
    """Zernike radial polynomial R_n^am(rho) by the factorial sum."""
    out = np.zeros_like(rho, dtype=np.float64)
    for s in range((n - am) // 2 + 1):
        coef = ((-1) ** s * factorial(n - s)
                / (factorial(s) * factorial((n + am) // 2 - s) * factorial((n - am) // 2 - s)))
        out = out + coef * rho ** (n - 2 * s)
    return out


def zernike(j, ky, kx, r):
    """Orthonormal Noll Zernike Z_j evaluated at integer frequency (ky, kx)."""
    ky = np.asarray(ky, dtype=np.float64)
    kx = np.asarray(kx, dtype=np.float64)
    n, m = noll_nm(j)
    rho = np.hypot(kx, ky) / r
    theta = np.arctan2(ky, kx)
    rad = radial(n, abs(m), rho)
    if m == 0:
        return np.sqrt(n + 1.0) * rad
    ang = np.cos(m * theta) if m > 0 else np.sin(-m * theta)
    return np.sqrt(2.0 * (n + 1)) * rad * ang


def pupil_phase(c, ky, kx, r):
    """phi(k) = sum_j c_j Z_j(k) over Noll j = 1..len(c) (c[0] is j = 1)."""
    c = np.asarray(c, dtype=np.float64)
    out = np.zeros(np.broadcast(np.asarray(ky), np.asarray(kx)).shape, dtype=np.float64)
    for idx, cj in enumerate(c):
        if cj != 0.0:
            out = out + cj * zernike(idx + 1, ky, kx, r)
    return out
