"""The seeded input module: LED lattice rule and the torch image formation,
checked against the oracle's own forward model."""

import numpy as np
import torch

import oracle
import apic_synth as S
from apic_synth.leds import led_ring


def test_led_lattice_examples():
    """Nearest lattice point on the ring, NA-matched LEDs inside the pupil."""
    ring = led_ring(128, 0.25, 8, 0.0, True)
    assert ring[:3] == [(24, 0), (17, 17), (0, 24)]
    ring = led_ring(256, 0.25, 16, 0.0, True)
    assert ring[:3] == [(49, 0), (45, 19), (35, 34)]
    r = 0.25 * 256 * 0.4 / 0.52
    assert all(x * x + y * y <= r * r for x, y in ring)
    df = led_ring(256, 0.38, 16, 0.5, False)
    assert all(x * x + y * y > r * r for x, y in df)


def test_config_sizes():
    w0 = S.single_tile()
    assert w0.n == 128 and len(w0.k_bf) == 8 and len(w0.k_df) == 8
    w1 = S.grid_batch(n_tiles=4)
    assert w1.n == 256 and len(w1.k_bf) == 16 and len(w1.k_df) == 32
    assert np.isclose(np.abs(S.field_model_quadratic(*np.meshgrid(
        (np.arange(32) - 15.5) / 15.5, (np.arange(32) - 15.5) / 15.5))[0]).max(), 1.5)


def test_torch_image_formation_matches_oracle_forward_model():
    w = S.small_workload(n=64, n_tiles=2)
    objs = np.stack([w.object(t) for t in range(2)])
    got = S.form_images(objs, w.coeffs, list(w.k_bf) + list(w.k_df), w.r).numpy()
    for t in range(2):
        want = oracle.forward_images(objs[t], list(w.k_bf) + list(w.k_df), w.coeffs[t], w.r)
        assert np.abs(got[t] - want).max() < 1e-12 * want.max()


def test_poisson_noise_scale():
    img = torch.full((4, 64, 64), 2.0, dtype=torch.float64)
    noisy = S.add_poisson(img, 1e4, seed=3)
    assert abs(noisy.mean().item() - 2.0) < 1e-3
    assert abs(noisy.var().item() - 2.0 / 1e4) < 2e-5


def test_slide_mask_and_scan_order():
    """The slide grid of 512 px tiles at 0.4 um is 122 x 371, the mask covers
    30% of it, the scan visits mask tiles in raster order, and the pool
    indices cycle through the tissue tiles with about 15% glass."""
    from apic_synth import slide
    assert slide.slide_grid() == (122, 371)
    m = slide.slide_mask()
    assert m.shape == (122, 371)
    assert abs(m.mean() - 0.30) < 1e-3
    idx, src = slide.scan_order(m, 400, 16, 4)
    assert np.all(np.diff(idx) > 0) and np.all(m.ravel()[idx])
    assert idx[0] == np.flatnonzero(m.ravel())[0]
    glass = src >= 16
    assert 0.08 < glass.mean() < 0.22
    assert np.array_equal(src[~glass], np.arange((~glass).sum()) % 16)
    assert np.all(src[glass] < 20)
    w = slide.pool_workload(16, 4)
    assert (w.n, w.n_bf, w.n_df, w.n_tiles) == (512, 16, 32, 20)
    assert np.abs(w.coeffs).max() <= 1.5 + 1e-9


def test_surrogate_workload_sets():
    """The surrogate workload's sets: 16384 training tiles of the uneven
    recipe without background or darkfield images at random positions, 4096
    evaluation tiles with 70% background and darkfield on the 64 x 64 grid;
    the two draw objects and noise from disjoint class seeds, and their pupils
    come from one field model (max 1.5 rad on the evaluation grid)."""
    import numpy as np
    tr = S.surrogate_train_batch()
    ev = S.surrogate_eval_batch()
    assert sum(w.n_tiles for w in tr) == 16384 and sum(w.n_tiles for w in ev) == 4096
    assert all(w.n_df == 0 and not w.extra["background"].any() for w in tr)
    assert all(w.n_df == 2 * w.n_bf for w in ev)
    assert sum(int(w.extra["background"].sum()) for w in ev) == round(0.7 * 4096)
    assert {w.seed_id for w in tr}.isdisjoint({w.seed_id for w in ev})
    sizes = np.concatenate([[w.n] * w.n_tiles for w in tr])
    assert (sizes == 128).sum() == 8192 and (sizes == 256).sum() == 6144
    pos = np.concatenate([w.positions for w in tr])
    assert np.all(np.abs(pos) <= 1.0) and len(np.unique(pos[:, 0])) == 16384
    c_ev = np.concatenate([w.coeffs for w in ev])
    assert abs(np.abs(c_ev).max() - 1.5) < 1e-12
    # the training pupils follow the same field model: evaluated at the
    # evaluation grid's positions they reproduce its coefficients
    w0 = ev[0]
    assert np.allclose(S.field_model_on_grid(w0.positions[:, 0], w0.positions[:, 1]), w0.coeffs)
