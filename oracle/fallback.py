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
the surrogate's prediction is used.  Sums re-wrapped about a seed c0 (the
seeded variant of Eq. 10) hold the system of the increment c - c0, so there
the residuals are those of the increments.
"""

import numpy as np


def residual(sums, c12):
    """R(c) from the normal-equation sums: expanding the square,
    sum w (beta - a.c)^2 = S_bb - 2 c.b + c.A c; divided by S_w."""
    c = np.asarray(c12, dtype=np.float64)
    A = np.asarray(sums["A"], dtype=np.float64)
    b = np.asarray(sums["b"], dtype=np.float64)
    return float((sums["sbb"] - 2.0 * (c @ b) + c @ A @ c) / sums["sw"])


def choose(sums, c_cf, c_sur, kappa, rho_max, kappa_max, resid_max, c0=None):
    """Returns (use_surrogate, rho, R(c_cf)) for Noll 4..15 candidates.

    When the sums were built with beta re-wrapped about a seed c0 (Noll
    4..15), they describe the increment over c0, and each candidate c is
    judged as R(c - c0)."""
    if c0 is not None:
        c0 = np.asarray(c0, dtype=np.float64)
        c_cf = np.asarray(c_cf, dtype=np.float64) - c0
        c_sur = np.asarray(c_sur, dtype=np.float64) - c0
    r_cf = residual(sums, c_cf)
    rho = float(np.sqrt(max(0.0, residual(sums, c_sur) - r_cf)))
    keep_cf = rho > rho_max and kappa <= kappa_max and r_cf <= resid_max
    return (not keep_cf), rho, r_cf
