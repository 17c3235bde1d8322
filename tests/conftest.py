import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side oracle runs")


@pytest.fixture(scope="session")
def lattice_geometry():
    """A lattice-exact geometry: N = 128 and r = 25 bins exactly (r^2 = 625 has
    20 lattice points), so NA-matched LEDs sit exactly on the pupil edge."""
    import numpy as np
    ring = [(25, 0), (20, 15), (15, 20), (0, 25), (-20, 15), (-25, 0), (-15, -20), (0, -25),
            (20, -15)]
    return {"n": 128, "dx_um": 0.390625, "wavelength_um": 0.5, "na_obj": 0.25,
            "k_bf": np.array(ring, dtype=np.int64)}


@pytest.fixture(autouse=True, scope="module")
def _release_cached_device_memory():
    """After each test module, hand the memory torch's caching allocator kept
    back to the device, so that a later module's own allocations (the slide
    streamer's staging buffers, the library's batch tables) find it free."""
    yield
    try:
        import gc
        import torch
        if torch.cuda.is_available():
            gc.collect()
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    except Exception:
        pass
