"""Pins of the oracle's colour combination (Sec. 3.3: amplitudes of the three
channel reconstructions, combined and white balanced).

* Channels of constant amplitudes a_R, a_G, a_B come out grey: every pixel
  equals the mean of the three, whatever the phases (the grey-world rule).
* Explicit gains multiply the amplitudes; the phase never enters.
* The grey-world gains of channels that differ by a constant factor undo it.
"""

import numpy as np

from oracle import rgb as orgb


def test_constant_channels_come_out_grey():
    a = (0.3, 0.8, 1.3)
    rng = np.random.default_rng(0)
    f = [a[c] * np.exp(1j * rng.uniform(-3, 3, (2, 4, 5))) for c in range(3)]
    img, g = orgb.combine(f)
    assert np.allclose(g, np.mean(a) / np.array(a), rtol=1e-14)
    assert img.shape == (2, 3, 4, 5)
    assert np.allclose(img, np.mean(a), rtol=1e-14)


def test_explicit_gains_and_phase_independence():
    rng = np.random.default_rng(1)
    amp = rng.uniform(0.1, 2.0, (3, 2, 6, 6))
    f1 = [amp[c] * np.exp(1j * rng.uniform(-3, 3, amp[c].shape)) for c in range(3)]
    f2 = [amp[c] + 0j for c in range(3)]
    g = (2.0, 0.5, 1.5)
    i1, _ = orgb.combine(f1, g)
    i2, _ = orgb.combine(f2, g)
    assert np.allclose(i1, i2, rtol=1e-14)
    assert np.allclose(i1[:, 1], 0.5 * amp[1], rtol=1e-14)


def test_grey_world_undoes_a_channel_scale():
    rng = np.random.default_rng(2)
    base = rng.uniform(0.2, 1.0, (3, 4, 4)) * np.exp(1j * rng.uniform(-1, 1, (3, 4, 4)))
    f = [base, 3.0 * base, 0.25 * base]
    img, g = orgb.combine(f)
    assert np.allclose(img[:, 0], img[:, 1], rtol=1e-13)
    assert np.allclose(img[:, 0], img[:, 2], rtol=1e-13)
