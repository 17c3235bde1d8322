"""Parity at the benchmark's full size and launch configuration: 1024 tiles of
256^2 (16 + 32 images, Poisson 1e4) reconstructed in one call, sampled tiles
checked against the FP64 oracle one by one."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import apic_synth as S
from apic_synth.batch import synth_batch
from paper_2407_20469_amd import apic
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_grid_batch_full_size_sampled_parity():
    w = S.grid_batch(n_tiles=1024)
    print("[gpu-test] synth 1024 grid tiles", flush=True)
    images = synth_batch(w, torch.device("cuda:0"))
    plan = apic.Plan(w.geometry_kwargs())
    print("[gpu-test] reconstruct 1024 grid tiles", flush=True)
    field, zern, status = apic.reconstruct(plan, images)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert not (st & (apic.TILE_NONFINITE_INPUT | apic.TILE_NONFINITE_OUT)).any()
    geom = oracle.Geometry(**w.geometry_kwargs())
    for t in (0, 613):
        ref = oracle.reconstruct(images[t].cpu().numpy().astype(np.float64), geom)
        err = rel_l2(field[t].cpu().numpy(), ref["field"])
        dz = float(np.abs(zern[t].cpu().numpy() - ref["c"]).max())
        print(f"[gpu-test] grid tile {t}: field rel-L2 {err:.3e} max|dc| {dz:.2e} "
              f"kappa {ref['pupil']['kappa']:.1f}", flush=True)
        assert dz < 1e-3
        assert err < 1e-4
