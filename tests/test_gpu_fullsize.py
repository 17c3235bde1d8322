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
from gpu_helpers import rel_l2, band_rel_l2

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
        f = field[t].cpu().numpy()
        err = rel_l2(f, ref["field"])
        err_df, err_bf = band_rel_l2(f, ref, geom)
        dz = float(np.abs(zern[t].cpu().numpy() - ref["c"]).max())
        print(f"[gpu-test] grid tile {t}: field rel-L2 {err:.3e} (darkfield band {err_df:.2e}, "
              f"brightfield band {err_bf:.2e}) max|dc| {dz:.2e} "
              f"kappa {ref['pupil']['kappa']:.1f}", flush=True)
        assert dz < 1e-3
        assert err < 1e-4
        assert err_df < 1e-3


@pytest.mark.timeout(900)
def test_grid_batch_with_surrogate_full_size():
    """The benchmark's timed configuration: the prepared batch of the 1024 grid
    tiles with the surrogate trained by the benchmark's recipe (closed-form
    estimates of training tiles disjoint from these) in the benchmark's mode,
    and autotuned chunks.  Every tile equals the plain surrogate call bit for
    bit; sampled tiles match the oracle given the coefficients the fallback
    rule chose, over the whole field and over the darkfield band."""
    import bench
    dev = torch.device("cuda:0")
    w = S.grid_batch(n_tiles=1024)
    print("[gpu-test] synth 1024 grid tiles", flush=True)
    images = synth_batch(w, dev)
    flat = images.reshape(-1)
    plan = apic.Plan(w.geometry_kwargs())
    plan.upload()
    print("[gpu-test] train the surrogate (benchmark recipe)", flush=True)
    sur, note = bench.train_grid_surrogate(w, dev)
    pos = torch.tensor(w.positions, dtype=torch.float32, device=dev)
    descs, n_img_el, n_fld_el = apic.mixed_descs(plan, np.zeros(w.n_tiles, np.int64))
    assert n_img_el == flat.numel()
    batch = apic.Batch(plan, descs)
    batch.set_surrogate(sur, pos)
    field = torch.empty(n_fld_el, dtype=torch.complex64, device=dev)
    zern = torch.empty((w.n_tiles, 15), dtype=torch.float32, device=dev)
    status = torch.empty((w.n_tiles,), dtype=torch.int32, device=dev)
    buf = torch.empty(batch.workspace_bytes + 256, dtype=torch.uint8, device=dev)
    print("[gpu-test] autotune and run the batch", flush=True)
    batch.autotune(flat, field, zern, status, (buf.data_ptr() + 255) & ~255,
                   batch.workspace_bytes, slack=0.0)
    del buf
    batch.reconstruct(flat, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    print("[gpu-test] plain surrogate call on the same tiles", flush=True)
    f_ref, z_ref, s_ref = apic.reconstruct_sur(plan, images, pos, sur)
    torch.cuda.synchronize()
    nf = w.n * w.upsample
    assert torch.equal(field.view(w.n_tiles, nf, nf), f_ref)
    assert torch.equal(zern, z_ref)
    assert torch.equal(status, s_ref)
    del f_ref
    st = status.cpu().numpy()
    used = int(((st & apic.TILE_SURROGATE_USED) != 0).sum())
    print(f"[gpu-test] surrogate kept on {used} of {w.n_tiles} tiles", flush=True)
    assert not (st & (apic.TILE_NONFINITE_INPUT | apic.TILE_NONFINITE_OUT)).any()
    assert np.all((st & (apic.TILE_SURROGATE_USED | apic.TILE_FALLBACK_USED)) != 0)
    geom = oracle.Geometry(**w.geometry_kwargs())
    fv = field.view(w.n_tiles, nf, nf)
    for t in (0, 613):
        zc = zern[t].cpu().numpy()
        ref = oracle.reconstruct(images[t].cpu().numpy().astype(np.float64), geom,
                                 zernike=zc.astype(np.float64))
        f = fv[t].cpu().numpy()
        err = rel_l2(f, ref["field"])
        err_df, _ = band_rel_l2(f, ref, geom)
        print(f"[gpu-test] grid tile {t} (status {int(st[t])}): field rel-L2 {err:.3e} "
              f"(darkfield band {err_df:.2e}) given the chosen coefficients", flush=True)
        assert err < 1e-4
        assert err_df < 1e-3
    batch.close()
