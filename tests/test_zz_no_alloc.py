"""The allocation-free entry point, apic_reconstruct_tiles_static, called
through the C ABI and compared with apic_reconstruct_tiles (caller workspace)
on the same tiles: two calls in a row, the second with fewer, different
tiles, so the static scratch still holds the first call's contents.  Also
its host-side refusals, which return before anything is enqueued.

Bar: the same kernels run on the same data with the same workspace layout,
so the outputs are expected to be identical; the test asserts field rel-L2
<= 1e-6 and Zernike within 1e-6 rad, and reports whether they are bit-equal.
"""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import apic_synth as S
from paper_2407_20469_amd import apic
from gpu_helpers import workload_images, rel_l2

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _log(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _static_call(plan, x, descs):
    T, n_img, n, _ = x.shape
    nf = 2 * n
    field = torch.full((T, nf, nf), complex(float("nan"), 0.0), dtype=torch.complex64, device=DEV)
    zern = torch.full((T, 15), float("nan"), dtype=torch.float32, device=DEV)
    status = torch.full((T,), -1, dtype=torch.int32, device=DEV)
    rc = plan.lib.apic_reconstruct_tiles_static(
        plan.handle, T, descs, apic._ptr(x), None, apic._ptr(zern), apic._ptr(field),
        apic._ptr(status), apic._stream(None))
    assert rc == apic.APIC_OK, apic.STATUS_NAMES.get(rc, rc)
    return field, zern, status


def test_static_scratch_matches_workspace_call():
    w = S.small_workload(n=128, n_bf=8, n_df=16, na_df=(0.30, 0.38), n_tiles=5, seed_id=53)
    imgs = workload_images(w, photons=1e4)
    plan = apic.Plan(w.geometry_kwargs())
    plan.upload()
    for label, sel in (("first call, 5 tiles", [0, 1, 2, 3, 4]), ("second call, 2 tiles", [4, 2])):
        x = torch.tensor(imgs[sel], device=DEV).contiguous()
        T, n_img, n, _ = x.shape
        descs = apic.tile_descs(T, n_img, n, 4 * n * n)
        _log(f"{label}: static scratch")
        f_s, z_s, s_s = _static_call(plan, x, descs)
        _log(f"{label}: caller workspace")
        f_w, z_w, s_w = apic.reconstruct(plan, x)
        torch.cuda.synchronize()
        f_s, f_w = f_s.cpu().numpy(), f_w.cpu().numpy()
        z_s, z_w = z_s.cpu().numpy(), z_w.cpu().numpy()
        for t in range(T):
            err = rel_l2(f_s[t], f_w[t])
            dz = float(np.abs(z_s[t] - z_w[t]).max())
            _log(f"  tile {sel[t]}: field rel-L2 {err:.2e}, max|dc| {dz:.2e}, "
                 f"bit-equal {np.array_equal(f_s[t], f_w[t]) and np.array_equal(z_s[t], z_w[t])}")
            assert err <= 1e-6 and dz <= 1e-6, sel[t]
        assert np.array_equal(s_s.cpu().numpy(), s_w.cpu().numpy())


def test_static_entry_refusals():
    """Host-side checks: a plan not uploaded to the device, a batch larger
    than the static array, an irregular descriptor list.  All return before
    any pointer is dereferenced or anything is enqueued."""
    w = S.small_workload(n=128, n_bf=8, n_df=16, na_df=(0.30, 0.38), n_tiles=1)
    n, n_img = w.n, w.n_img
    fake = ctypes.c_void_p(1 << 20)
    stream = apic._stream(None)
    fresh = apic.Plan(w.geometry_kwargs())
    descs = apic.tile_descs(1, n_img, n, 4 * n * n)
    rc = fresh.lib.apic_reconstruct_tiles_static(fresh.handle, 1, descs, fake, None, fake, fake,
                                                 fake, stream)
    assert rc == apic.APIC_EPLAN
    plan = apic.Plan(w.geometry_kwargs())
    plan.upload()
    per_tile = plan.workspace_bytes(apic.tile_descs(1, n_img, n, 4 * n * n))
    many = (256 << 20) // per_tile + 1
    descs = apic.tile_descs(many, n_img, n, 4 * n * n)
    rc = plan.lib.apic_reconstruct_tiles_static(plan.handle, many, descs, fake, None, fake, fake,
                                                fake, stream)
    assert rc == apic.APIC_ENOMEM
    descs = apic.tile_descs(3, n_img, n, 4 * n * n)
    descs[1].image_offset, descs[2].image_offset = descs[2].image_offset, descs[1].image_offset
    rc = plan.lib.apic_reconstruct_tiles_static(plan.handle, 3, descs, fake, None, fake, fake,
                                                fake, stream)
    assert rc == apic.APIC_EUNSUPPORTED
    _log(f"refusals checked ({many} tiles of {per_tile / 2 ** 20:.1f} MiB exceed the array)")
