"""Pins of the surrogate fallback rule in the oracle (oracle/fallback.py):
the residual from normal-equation sums against brute force over explicit rows,
the closed-form solution as the residual's minimiser, and the decision at its
thresholds."""

import numpy as np
import pytest

from oracle import fallback as FB


def _rows(seed, m=200):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.1, 2.0, m)
    a = rng.standard_normal((m, 12))
    beta = a @ rng.normal(0, 0.3, 12) + rng.normal(0, 0.05, m)
    sums = {"A": (a * w[:, None]).T @ a, "b": (w * beta) @ a, "sbb": float(w @ beta ** 2),
            "sw": float(w.sum())}
    return w, a, beta, sums


def test_residual_matches_brute_force_over_rows():
    w, a, beta, sums = _rows(1)
    rng = np.random.default_rng(2)
    for _ in range(5):
        c = rng.normal(0, 0.5, 12)
        brute = float(np.sum(w * (beta - a @ c) ** 2) / w.sum())
        assert abs(FB.residual(sums, c) - brute) < 1e-12 * max(1.0, brute)


def test_least_squares_solution_minimises_the_residual():
    w, a, beta, sums = _rows(3)
    sw = np.sqrt(w)
    c_ls = np.linalg.lstsq(a * sw[:, None], beta * sw, rcond=None)[0]
    r0 = FB.residual(sums, c_ls)
    rng = np.random.default_rng(4)
    for _ in range(20):
        assert FB.residual(sums, c_ls + rng.normal(0, 1e-2, 12)) >= r0
    use_sur, rho, r_cf = FB.choose(sums, c_ls, c_ls, 1.0, 0.0, 1e6, 1e6)
    assert rho == 0.0 and r_cf == r0 and use_sur  # rho = 0 is not above rho_max = 0


def test_decision_at_the_thresholds():
    w, a, beta, sums = _rows(5)
    sw = np.sqrt(w)
    c_ls = np.linalg.lstsq(a * sw[:, None], beta * sw, rcond=None)[0]
    c_far = c_ls + 0.2
    _, rho, r_cf = FB.choose(sums, c_ls, c_far, 10.0, 0.0, 1e6, 1e6)
    # rho^2 is the excess residual, a quadratic form in the difference
    d = c_far - c_ls
    assert abs(rho ** 2 - d @ sums["A"] @ d / sums["sw"]) < 1e-10 * rho ** 2
    assert FB.choose(sums, c_ls, c_far, 10.0, rho * 1.001, 1e6, 1e6)[0]       # within rho_max
    assert not FB.choose(sums, c_ls, c_far, 10.0, rho * 0.999, 1e6, 1e6)[0]   # too far: closed form
    assert FB.choose(sums, c_ls, c_far, 10.0, rho * 0.999, 5.0, 1e6)[0]       # ill-conditioned
    assert FB.choose(sums, c_ls, c_far, 10.0, rho * 0.999, 1e6, r_cf * 0.5)[0]  # poor fit
