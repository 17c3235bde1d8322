"""Pins of the oracle's background-tile statistic (Sec. 3.2: patches whose
low-resolution images vary less than a threshold are skipped).

Each check compares the oracle with a value worked out by hand or a closed
form, so a sample-variance divisor, a missing square of the mean, pooling the
images instead of averaging them, or reading the darkfield images would fail.
"""

import numpy as np
import pytest
import torch

from oracle import background as obg


def test_hand_worked_2x2():
    """[[1, 2], [3, 4]]: mean 5/2, population variance 5/4, statistic 1/5."""
    assert obg.relative_variance(np.array([[1.0, 2.0], [3.0, 4.0]])) == pytest.approx(0.2, rel=1e-15)


@pytest.mark.parametrize("n,p,q,a", [(8, 1, 0, 0.3), (8, 2, 3, 0.5), (16, 5, 7, 0.1)])
def test_cosine_closed_form(n, p, q, a):
    """m (1 + a cos(2 pi (p x + q y) / n)) has mean m and population variance
    m^2 a^2 / 2 over the full period, so the statistic is a^2 / 2; at n = 8 a
    sample-variance divisor would be off by 64/63."""
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    img = 3.7 * (1.0 + a * np.cos(2 * np.pi * (p * x + q * y) / n))
    assert obg.relative_variance(img) == pytest.approx(a * a / 2, rel=1e-12)


def test_two_level_image():
    """Half the pixels at u, half at v: statistic ((u - v) / (u + v))^2."""
    u, v = 0.8, 1.3
    img = np.full((6, 6), u)
    img[:, 3:] = v
    assert obg.relative_variance(img) == pytest.approx(((u - v) / (u + v)) ** 2, rel=1e-13)


def test_mean_over_na_matched_images_only():
    """The tile statistic averages the per-image values of the first n_bf
    images; darkfield images (here with a huge variance) do not enter, and
    images of different brightness are not pooled."""
    n = 8
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a1, a2 = 0.2, 0.6
    i1 = 1.0 * (1 + a1 * np.cos(2 * np.pi * x / n))
    i2 = 9.0 * (1 + a2 * np.cos(2 * np.pi * y / n))
    dfi = np.zeros((n, n))
    dfi[0, 0] = 1e6
    stack = np.stack([i1, i2, dfi, dfi])
    want = (a1 * a1 / 2 + a2 * a2 / 2) / 2
    assert obg.background_stat(stack, 2) == pytest.approx(want, rel=1e-12)
    pooled = np.mean((stack[:2] - stack[:2].mean()) ** 2) / stack[:2].mean() ** 2
    assert abs(pooled - want) > 0.1 * want


def test_scale_invariance_and_constant():
    rng = np.random.default_rng(0)
    img = rng.uniform(0.5, 1.5, (12, 12))
    assert obg.relative_variance(7.0 * img) == pytest.approx(obg.relative_variance(img), rel=1e-13)
    assert obg.relative_variance(np.full((4, 4), 2.5)) == 0.0


def test_separates_glass_from_tissue():
    """On synthetic 128 px tiles at 1e4 photons, near-empty glass stays well
    under 1e-3 and blob tissue well over 1e-2 (the threshold range the
    stream uses)."""
    from apic_synth.configs import Workload, uneven_classes, field_model_quadratic
    from apic_synth.objects import object_background, object_blobs
    from apic_synth.imaging import form_images, add_poisson
    cls = uneven_classes()[0]
    w = Workload("t", cls["n"], cls["k_bf"], cls["k_df"])
    c, _ = field_model_quadratic(np.zeros(1), np.zeros(1))
    stats = {}
    for name, fn in (("glass", object_background), ("tissue", object_blobs)):
        o = fn(np.random.default_rng([5, 0, 1]), w.n)[None]
        im = form_images(o, c, [tuple(k) for k in w.k_bf], w.r, dtype=torch.float64)
        im = add_poisson(im, 1e4, seed=3)[0].numpy()
        stats[name] = obg.background_stat(im, w.n_bf)
    assert stats["glass"] < 1e-3 < 1e-2 < stats["tissue"]
