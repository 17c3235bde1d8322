"""The tile batcher on the GPU: an uneven batch of three geometry classes
(64^2 with 8 + 8 images, 64^2 with 12 + 12 on two darkfield rings, 128^2 with
8 + 16), interleaved in memory and with one tile flagged to skip the darkfield
stage, run through the prepared batch (descriptors on the device, classes on
concurrent side streams) and through a captured graph replayed several times.

Bars: the batch and every graph replay reproduce the plain call on the same
descriptors exactly (same kernels, fixed reduction orders); one tile of each
class is checked against the FP64 oracle at field rel-L2 1e-4 and Noll
coefficients 1e-3 rad.
"""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import apic_synth as S
from paper_2407_20469_amd import apic
from gpu_helpers import oracle_geometry, rel_l2, workload_images, band_rel_l2

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def uneven():
    ws = [S.small_workload(n=64, n_bf=8, n_df=8, n_tiles=3, seed_id=21),
          S.small_workload(n=64, n_bf=12, n_df=12, na_df=(0.30, 0.32), n_tiles=2, seed_id=22),
          S.small_workload(n=128, n_bf=8, n_df=16, na_df=(0.30, 0.38), n_tiles=2, seed_id=23)]
    imgs = [workload_images(w) for w in ws]
    # interleaved tile order: (class, tile within class); the last tile skips darkfield
    order = [(0, 0), (2, 0), (1, 0), (0, 1), (2, 1), (1, 1), (0, 2)]
    flags = [0] * (len(order) - 1) + [apic.TILE_SKIP_DARKFIELD]
    plan = apic.Plan([w.geometry_kwargs() for w in ws])
    descs, n_img_el, n_fld_el = apic.mixed_descs(plan, [c for c, _ in order], flags)
    flat = np.concatenate([imgs[c][t].ravel() for c, t in order]).astype(np.float32)
    assert flat.size == n_img_el
    return ws, imgs, order, flags, plan, descs, n_fld_el, torch.tensor(flat, device=DEV)


def _buffers(n_tiles, n_fld_el):
    field = torch.full((n_fld_el,), float("nan"), dtype=torch.complex64, device=DEV)
    zern = torch.full((n_tiles, 15), float("nan"), dtype=torch.float32, device=DEV)
    status = torch.full((n_tiles,), -1, dtype=torch.int32, device=DEV)
    return field, zern, status


def _plain(plan, descs, images, n_fld_el):
    field, zern, status = _buffers(len(descs), n_fld_el)
    ws = apic.Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), images.device)
    code = plan.lib.apic_reconstruct_tiles(plan.handle, len(descs), descs, apic._ptr(images), None,
                                           apic._ptr(zern), apic._ptr(field), apic._ptr(status),
                                           wp, wb, apic._stream(None))
    assert code == apic.APIC_OK
    torch.cuda.synchronize()
    return field.cpu().numpy(), zern.cpu().numpy(), status.cpu().numpy()


def test_batch_matches_plain_and_oracle(uneven):
    ws_, imgs, order, flags, plan, descs, n_fld_el, images = uneven
    _log(f"uneven batch of {len(order)} tiles over 3 classes")
    ref_f, ref_z, ref_s = _plain(plan, descs, images, n_fld_el)
    batch = apic.Batch(plan, descs)
    field, zern, status = _buffers(len(descs), n_fld_el)
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    f, z, st = field.cpu().numpy(), zern.cpu().numpy(), status.cpu().numpy()
    assert np.array_equal(f, ref_f)
    assert np.array_equal(z, ref_z)
    assert np.array_equal(st, ref_s)
    # oracle: the first tile of each class and the skip tile
    seen = set()
    for t, (c, i) in enumerate(order):
        if c in seen and flags[t] == 0:
            continue
        seen.add(c)
        w = ws_[c]
        g = oracle_geometry(w)
        ref = oracle.reconstruct(imgs[c][i], g)
        want = ref["field"] if flags[t] == 0 else oracle.upsampled_field(ref["bf_hat"], w.upsample)
        nf = w.n * w.upsample
        d = descs[t]
        got = f[d.field_offset:d.field_offset + nf * nf].reshape(nf, nf)
        err = rel_l2(got, want)
        dz = np.abs(z[t] - ref["c"]).max()
        _log(f"tile {t} (class {c}, flags {flags[t]}): field rel-L2 {err:.2e}  max|dc| {dz:.1e}")
        assert err < 1e-4
        assert dz < 1e-3
    batch.close()


def test_graph_replay_matches_eager(uneven):
    ws_, imgs, order, flags, plan, descs, n_fld_el, images = uneven
    batch = apic.Batch(plan, descs)
    stream = torch.cuda.Stream()
    work = images.clone()
    field, zern, status = _buffers(len(descs), n_fld_el)
    wsp = apic.Workspace()
    wsp.get(batch.workspace_bytes, images.device)  # allocate before capture
    torch.cuda.synchronize()
    _log("capture")
    batch.capture(work, field, zern, status, wsp, stream)
    torch.cuda.synchronize()
    gen = torch.Generator(device=DEV)
    gen.manual_seed(3)
    for rep in range(3):
        # new contents in the bound input buffer: scaled intensities (the method is
        # invariant to a global scale up to rounding) plus small positive noise
        with torch.cuda.stream(stream):
            scale = 0.5 + rep
            work.copy_(images * scale + 1e-4 * torch.rand(images.shape, generator=gen,
                                                          device=DEV))
            field.fill_(float("nan"))
            batch.launch(stream)
        stream.synchronize()
        got = (field.cpu().numpy(), zern.cpu().numpy(), status.cpu().numpy())
        eager_f, eager_z, eager_s = _buffers(len(descs), n_fld_el)
        batch.reconstruct(work, eager_f, eager_z, eager_s, apic.Workspace())
        torch.cuda.synchronize()
        _log(f"replay {rep}: max|field diff| "
             f"{np.abs(got[0] - eager_f.cpu().numpy()).max():.2e}")
        assert np.array_equal(got[0], eager_f.cpu().numpy())
        assert np.array_equal(got[1], eager_z.cpu().numpy())
        assert np.array_equal(got[2], eager_s.cpu().numpy())
    batch.close()


def test_fft_panel_variants_give_identical_results(uneven):
    """Every class with the alternative panel width of its FFT column passes
    (the autotuner's LDS-tiling choice) reproduces the plain call bit for bit:
    each column's transform is the same, only the access pattern changes."""
    _, _, _, _, plan, descs, n_fld_el, images = uneven
    ref_f, ref_z, ref_s = _plain(plan, descs, images, n_fld_el)
    batch = apic.Batch(plan, descs)
    before = batch.classes()
    for i in range(len(before)):
        batch.set_fft(i, 1)
    after = batch.classes()
    _log("panel columns per class: " + ", ".join(
        f"{b['fft_panel_columns']} -> {a['fft_panel_columns']}" for b, a in zip(before, after)))
    assert all(a["fft_variant"] == 1 for a in after)
    assert any(a["fft_panel_columns"] != b["fft_panel_columns"] for a, b in zip(after, before))
    field, zern, status = _buffers(len(descs), n_fld_el)
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    assert np.array_equal(field.cpu().numpy(), ref_f)
    assert np.array_equal(zern.cpu().numpy(), ref_z)
    assert np.array_equal(status.cpu().numpy(), ref_s)
    with pytest.raises(apic.ApicError):
        batch.set_fft(0, 2)
    batch.close()


def test_batch_rejects_bad_descriptors(uneven):
    _, _, _, _, plan, descs, _, _ = uneven
    bad = (apic.TileDesc * 1)()
    bad[0].geom = 7
    with pytest.raises(apic.ApicError):
        apic.Batch(plan, bad)
    empty = apic.Batch(plan, (apic.TileDesc * 0)())
    assert empty.workspace_bytes >= 0
    empty.close()


def test_chunked_and_autotuned_batch_match_plain(uneven):
    _, _, _, _, plan, descs, n_fld_el, images = uneven
    ref_f, ref_z, ref_s = _plain(plan, descs, images, n_fld_el)
    batch = apic.Batch(plan, descs)
    full_ws = batch.workspace_bytes
    classes = batch.classes()
    _log(f"classes {classes}")
    assert sum(c["n_tiles"] for c in classes) == len(descs)
    for i in range(len(classes)):
        batch.set_chunk(i, 1)
    assert batch.workspace_bytes < full_ws
    field, zern, status = _buffers(len(descs), n_fld_el)
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    assert np.array_equal(field.cpu().numpy(), ref_f)
    assert np.array_equal(zern.cpu().numpy(), ref_z)
    assert np.array_equal(status.cpu().numpy(), ref_s)
    # one-tile chunks on two lanes (two streams per class, two chunk workspaces)
    for i in range(len(classes)):
        batch.set_chunk(i, 1, lanes=2)
    field, zern, status = _buffers(len(descs), n_fld_el)
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    assert np.array_equal(field.cpu().numpy(), ref_f)
    assert np.array_equal(zern.cpu().numpy(), ref_z)
    assert np.array_equal(status.cpu().numpy(), ref_s)
    # autotune within the whole-batch workspace, then run with the chosen chunks
    buf = torch.empty(full_ws + 256, dtype=torch.uint8, device=DEV)
    wp = (buf.data_ptr() + 255) & ~255
    ms = batch.autotune(images, field, zern, status, wp, full_ws)
    chosen = [c["chunk"] for c in batch.classes()]
    _log(f"autotuned chunks {chosen}, ms per tile {np.round(ms, 3).tolist()}")
    assert np.all(ms > 0)
    for c, k in zip(batch.classes(), chosen):
        assert 1 <= k <= c["n_tiles"]
    field, zern, status = _buffers(len(descs), n_fld_el)
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    assert np.array_equal(field.cpu().numpy(), ref_f)
    assert np.array_equal(status.cpu().numpy(), ref_s)
    batch.close()


def _const_surrogate(c_const):
    """A surrogate whose weights are all zero, so that it predicts the output
    bias: Noll coefficients 4..15 = c_const on every tile."""
    theta = np.zeros_like(apic.init_mlp_params(0))
    b3 = 128 * 64 + 128 + 128 * 128 + 128 + 16 * 128
    assert theta.size == b3 + 16
    theta[b3:b3 + 12] = c_const
    return apic.Surrogate(theta, np.zeros(34), np.ones(34), device=DEV)


def _plain_sur(plan, descs, images, n_fld_el, pos, sur, rho_max):
    field, zern, status = _buffers(len(descs), n_fld_el)
    ws = apic.Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), images.device)
    mdl = sur.model()
    code = plan.lib.apic_reconstruct_tiles_sur(
        plan.handle, len(descs), descs, apic._ptr(images), apic._ptr(pos), ctypes.byref(mdl),
        float(rho_max), 1e6, 1.0, apic._ptr(zern), apic._ptr(field), apic._ptr(status), wp, wb,
        apic._stream(None))
    assert code == apic.APIC_OK
    torch.cuda.synchronize()
    return field.cpu().numpy(), zern.cpu().numpy(), status.cpu().numpy()


def test_batch_with_surrogate(uneven):
    """The prepared batch with the surrogate and its fallback rule: eager, on
    two lanes it reproduces apic_reconstruct_tiles_sur on the same
    descriptors exactly; with the surrogate forced on every tile
    the fields match the oracle given the chosen coefficients (field rel-L2
    1e-4); switching the surrogate off restores the plain batch."""
    ws_, imgs, order, flags, plan, descs, n_fld_el, images = uneven
    rng = np.random.default_rng(41)
    c_const = rng.uniform(-0.1, 0.1, 12).astype(np.float32)
    sur = _const_surrogate(c_const)
    pos = torch.tensor(rng.uniform(-1, 1, (len(descs), 2)), dtype=torch.float32, device=DEV)
    batch = apic.Batch(plan, descs)
    for rho_max in (1e30, 0.05):
        _log(f"batch + surrogate, rho_max {rho_max:g}")
        ref_f, ref_z, ref_s = _plain_sur(plan, descs, images, n_fld_el, pos, sur, rho_max)
        batch.set_surrogate(sur, pos, rho_max=rho_max)
        for lanes in (1, 2):
            for i in range(len(batch.classes())):
                batch.set_chunk(i, 1 if lanes == 2 else 0, lanes=lanes)
            field, zern, status = _buffers(len(descs), n_fld_el)
            batch.reconstruct(images, field, zern, status, apic.Workspace())
            torch.cuda.synchronize()
            assert np.array_equal(field.cpu().numpy(), ref_f)
            assert np.array_equal(zern.cpu().numpy(), ref_z)
            assert np.array_equal(status.cpu().numpy(), ref_s)
        used = (ref_s & apic.TILE_SURROGATE_USED) != 0
        _log(f"  surrogate kept on {int(used.sum())} of {len(descs)} tiles")
        if rho_max > 1:
            assert used.all()
            assert np.array_equal(ref_z[:, 3:], np.broadcast_to(c_const, (len(descs), 12)))
            for t, (c, i) in enumerate(order):
                if flags[t]:
                    continue
                w = ws_[c]
                ref = oracle.reconstruct(imgs[c][i], oracle_geometry(w),
                                         zernike=ref_z[t].astype(np.float64))
                nf = w.n * w.upsample
                d = descs[t]
                got = ref_f[d.field_offset:d.field_offset + nf * nf].reshape(nf, nf)
                err = rel_l2(got, ref["field"])
                _log(f"  tile {t} (class {c}): field rel-L2 {err:.2e} vs oracle")
                assert err < 1e-4
        else:
            assert (~used).any()  # the constant guess is far off on these tiles
    # graphs are offered for one-lane batches without the surrogate only: the
    # refusal comes from the host before any capture starts
    stream = torch.cuda.Stream()
    field, zern, status = _buffers(len(descs), n_fld_el)
    with pytest.raises(apic.ApicError):
        batch.capture(images, field, zern, status, apic.Workspace(), stream)
    # surrogate off: the plain batch again
    batch.set_surrogate(None, None)
    plain_f, plain_z, _ = _plain(plan, descs, images, n_fld_el)
    field, zern, status = _buffers(len(descs), n_fld_el)
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    assert np.array_equal(field.cpu().numpy(), plain_f)
    assert np.array_equal(zern.cpu().numpy(), plain_z)
    batch.close()


def _synth_flat(ws, geom_ids, tile_ids):
    """Flat float32 images of the given (class, tile) list, synthesised on the GPU."""
    from apic_synth.batch import synth_batch
    parts = []
    for c, t in zip(geom_ids, tile_ids):
        parts.append(synth_batch(ws[c], DEV, tiles=[t]).reshape(-1))
    return torch.cat(parts)


@pytest.mark.timeout(900)
def test_uneven_nine_class_batch():
    """One tile of each of the nine classes of the uneven batch (128/256/512 px x
    8/12/16 NA-matched LEDs, twice as many darkfield), background and content
    tiles, Poisson noise: the autotuned concurrent batch equals the plain call,
    and every class's tile matches the FP64 oracle (the full chain, every
    darkfield image; the T - E route of the oracle's gram from 256 px on):
    field rel-L2 1e-4, darkfield band 1e-3, Zernike 1e-3 rad."""
    ws = S.uneven_batch(n_tiles=4096)
    plan = apic.Plan([w.geometry_kwargs() for w in ws])
    geom_ids = list(range(len(ws)))
    tile_ids = [int(np.argmax(w.extra["background"])) if c % 2 else 0
                for c, w in enumerate(ws)]
    _log(f"nine-class batch: tiles {tile_ids}")
    images = _synth_flat(ws, geom_ids, tile_ids)
    descs, n_img_el, n_fld_el = apic.mixed_descs(plan, geom_ids)
    assert images.numel() == n_img_el
    ref_f, ref_z, ref_s = _plain(plan, descs, images, n_fld_el)
    batch = apic.Batch(plan, descs)
    field, zern, status = _buffers(len(descs), n_fld_el)
    buf = torch.empty(batch.workspace_bytes + 256, dtype=torch.uint8, device=DEV)
    batch.autotune(images, field, zern, status, (buf.data_ptr() + 255) & ~255,
                   batch.workspace_bytes)
    del buf
    field, zern, status = _buffers(len(descs), n_fld_el)
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    f = field.cpu().numpy()
    assert np.array_equal(f, ref_f)
    assert np.array_equal(zern.cpu().numpy(), ref_z)
    assert np.array_equal(status.cpu().numpy(), ref_s)
    assert np.all(np.isfinite(f))
    z = zern.cpu().numpy()
    for c in range(len(ws)):
        w = ws[c]
        d = descs[c]
        img = images[d.image_offset:d.image_offset + w.n_img * w.n * w.n]
        img = img.reshape(w.n_img, w.n, w.n).cpu().numpy()
        geom = oracle_geometry(w)
        ref = oracle.reconstruct(img, geom, gram="t-e" if w.n >= 256 else "fullq")
        nf = w.n * w.upsample
        fc = f[d.field_offset:d.field_offset + nf * nf].reshape(nf, nf)
        err = rel_l2(fc, ref["field"])
        err_df, _ = band_rel_l2(fc, ref, geom)
        dz = np.abs(z[c] - ref["c"]).max()
        _log(f"class {c} ({w.n} px, {w.n_bf}+{w.n_df}, tile {tile_ids[c]}): field rel-L2 "
             f"{err:.2e} (darkfield band {err_df:.2e}) max|dc| {dz:.1e}")
        assert err < 1e-4
        assert err_df < 1e-3
        assert dz < 1e-3
    batch.close()


@pytest.mark.timeout(900)
def test_512_tile_with_one_darkfield_image():
    """A 512 px tile (16 NA-matched LEDs of the uneven batch's largest class and
    its first darkfield LED) against the oracle: the largest unknown count of
    the batch (N_u of the first darkfield image)."""
    ws = S.uneven_batch(n_tiles=4096)
    big = ws[8]
    w = S.Workload("512-16+1", big.n, big.k_bf, big.k_df[:1], upsample=2, n_tiles=1,
                   photons=1e4, seed_id=big.seed_id, coeffs=big.coeffs[:1],
                   positions=big.positions[:1])
    plan = apic.Plan(w.geometry_kwargs())
    _log(f"512 px tile: plan sizes {plan.sizes()}")
    from apic_synth.batch import synth_batch
    imgs = synth_batch(w, DEV)
    field, z, status = apic.reconstruct(plan, imgs)
    torch.cuda.synchronize()
    ref = oracle.reconstruct(imgs[0].cpu().numpy(), oracle_geometry(w))
    err = rel_l2(field[0].cpu().numpy(), ref["field"])
    dz = np.abs(z[0].cpu().numpy() - ref["c"]).max()
    info = ref["darkfield"][0]
    _log(f"512 px: N_u {info.get('n_u')}, field rel-L2 {err:.2e}, max|dc| {dz:.1e}, "
         f"status {int(status[0])}")
    assert err < 1e-4
    assert dz < 1e-3
