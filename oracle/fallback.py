"""Choice between the learned surrogate's pupil and the closed-form solve of
Eq. 10 (the surrogate is not in the paper; the closed form judges it).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading taken: with the Eq. 10 system of a tile reduced to its normal-equation
sums, A = sum w a a^T, b = sum w beta a, S_bb = sum w beta^2 and S_w = sum w
over the rows (w, beta, a), the weighted linearised residual of coefficients c
(Noll 4..15) is R(c) = sum w (beta - a.c)^2 / S_w.  The surrogate's
prediction c_s costs rho = sqrt(max(0, R(c_s) - R(c_cf))) over the closed-form
c_cf.  The closed form is kept when rho > rho_max while it is trustworthy
(condition number kappa(A) <= kappa_max and R(c_cf) <= resid_max); otherwise
the surrogate's prediction is used.
"""

import numpy as np


def residual(sums, c12):
    """R(c) from the normal-equation sums: expanding the square,
    sum w (beta - a.c)^2 = S_bb - 2 c.b + c.A c; divided by S_w."""
    c = np.asarray(c12, dtype=np.float64)
    A = np.asarray(sums["A"], dtype=np.float64)
    b = np.asarray(sums["b"], dtype=np.float64)
    return float((sums["sbb"] - 2.0 * (c @ b) + c @ A @ c) / sums["sw"])


def choose(sums, c_cf, c_sur, kappa, rho_max, kappa_max, resid_max):
    """Returns (use_surrogate, rho, R(c_cf)) for Noll 4..15 candidates."""
    r_cf = residual(sums, c_cf)
    rho = float(np.sqrt(max(0.0, residual(sums, c_sur) - r_cf)))
    keep_cf = rho > rho_max and kappa <= kappa_max and r_cf <= resid_max
    return (not keep_cf), rho, r_cf
