"""Host logic of the C ABI, on the CPU: the plan's index tables equal the
oracle's sets bit for bit; every symbol declared in include/apic.h is exported;
argument errors are rejected before anything is enqueued."""

import ctypes
import os
import re

import numpy as np

from oracle import aberration as oab
import pytest

import oracle
from oracle import darkfield as odf
from oracle.aberration import pupil_pairs, feature_cell
from oracle.grid import k_grid, circ
import apic_synth as S
from paper_2407_20469_amd import apic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "apic.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apic_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = apic.load_library()
    declared = _declared_functions()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(apic.EXPORTS)
    assert b"gfx950" in lib.apic_version()


@pytest.mark.parametrize("wl", ["single128", "small64", "two_ring128", "grid256", "slide512"])
def test_plan_sets_equal_oracle_sets(wl):
    """Also at the two benchmark geometries: 256 px and 512 px, 16 NA-matched
    and 32 darkfield images on two rings."""
    if wl == "single128":
        w = S.single_tile()
    elif wl == "small64":
        w = S.small_workload(n=64)
    elif wl == "grid256":
        w = S.grid_batch()
    elif wl == "slide512":
        from apic_synth import slide
        w = slide.pool_workload(2, 1)
    else:
        w = S.small_workload(n=128, n_bf=12, n_df=24, na_df=(0.30, 0.38))
    plan = apic.Plan(w.geometry_kwargs())
    n, r = w.n, w.r
    ky, kx = k_grid(n)
    known = np.zeros((n, n), bool)
    for k in w.k_bf:
        known |= circ(ky + k[1], kx + k[0], r)
    for j, k_j in enumerate(w.k_df):
        sets = odf.darkfield_sets(n, k_j, known, r)
        for what, key in enumerate(["U", "P", "Q", "E"]):
            got = plan.query(what, 0, j).reshape(-1, 2)
            want = sets[key] if len(sets["U"]) or key in ("U", "P") else np.zeros((0, 2))
            want = np.asarray(want).reshape(-1, 2)
            # the plan may order U and E for locality: compare as sets, no repeats
            assert len(got) == len(want), (j, key)
            assert np.array_equal(got[np.lexsort(got.T[::-1])], want[np.lexsort(want.T[::-1])]), \
                (j, key)
        known |= sets["U_mask"]
    rows = plan.query(4).reshape(-1, 5)
    want = []
    for i, l, K_y, K_x in pupil_pairs(n, w.k_bf, r):
        cells = feature_cell(w.k_bf[i], w.k_bf[l], K_y, K_x, r)
        for a, b, c in zip(K_y, K_x, cells):
            want.append((i, l, a, b, c))
    want = np.array(want)
    # the same rows (the plan sorts them by continuation band)
    assert len(rows) == len(want)
    assert np.array_equal(rows[np.lexsort(rows.T[::-1])], want[np.lexsort(want.T[::-1])])
    # each band pass is a prefix of the plan's rows: the oracle's rows with
    # |K| <= f r, counted by the oracle's own band selection
    ones = np.ones((len(w.k_bf), n, n), complex)
    counts = [oab.aberration_sums(ones, w.k_bf, r, k_max=f * r)["rows"] for f in oab.PUPIL_BANDS]
    want_bands = [c for c in counts if c >= oab.MIN_BAND_ROWS]
    got_bands = list(plan.query(7))
    assert got_bands == want_bands
    k2 = rows[:, 2].astype(np.float64) ** 2 + rows[:, 3].astype(np.float64) ** 2
    for f, cnt in zip(oab.PUPIL_BANDS, counts):
        inside = k2 <= (f * r) ** 2
        assert inside.sum() == cnt and np.all(inside[:cnt])


@pytest.mark.parametrize("wl", ["small64", "two_ring128", "grid256", "slide512"])
def test_plan_row_spans_cover_every_read(wl):
    """The darkfield FFT passes skip rows (Eq. 11-13 chain): P_hat and U lie on
    the rows of P + U, b on the rows of Q, and fft2(|P|^2 + i I_j) is read on
    Q, on -Q and at the row differences of U. Each span the plan reports is
    the exact extent of the oracle's sets."""
    if wl == "small64":
        w = S.small_workload(n=64)
    elif wl == "grid256":
        w = S.grid_batch()
    elif wl == "slide512":
        from apic_synth import slide
        w = slide.pool_workload(2, 1)
    else:
        w = S.small_workload(n=128, n_bf=12, n_df=24, na_df=(0.30, 0.38))
    plan = apic.Plan(w.geometry_kwargs())
    spans = plan.query(8).reshape(-1, 6)
    assert spans.shape[0] == len(w.k_df)
    n, r = w.n, w.r
    ky, kx = k_grid(n)
    known = np.zeros((n, n), bool)
    for k in w.k_bf:
        known |= circ(ky + k[1], kx + k[0], r)
    executed = 0
    for j, k_j in enumerate(w.k_df):
        sets = odf.darkfield_sets(n, k_j, known, r)
        known |= sets["U_mask"]
        d_lo, d_hi, q_lo, q_hi, z_lo, z_hi = spans[j].tolist()
        u = np.asarray(sets["U"]).reshape(-1, 2)
        if len(u) == 0:
            assert (d_lo, d_hi, q_lo, q_hi, z_lo, z_hi) == (0, -1, 0, -1, 0, -1), j
            continue
        executed += 1
        pu_rows = np.concatenate([np.asarray(sets["P"]).reshape(-1, 2)[:, 0], u[:, 0]])
        assert (d_lo, d_hi) == (pu_rows.min(), pu_rows.max()), j
        q_rows = np.asarray(sets["Q"]).reshape(-1, 2)[:, 0]
        w_u = int(u[:, 0].max() - u[:, 0].min())
        read = [np.arange(-w_u, w_u + 1)]  # row differences of U, both signs
        if len(q_rows):
            assert (q_lo, q_hi) == (q_rows.min(), q_rows.max()), j
            read += [q_rows, -q_rows]
        else:
            assert (q_lo, q_hi) == (0, -1), j
        read = np.concatenate(read)
        assert (z_lo, z_hi) == (read.min(), read.max()), j
        # every span fits the grid without wrapping onto itself
        assert d_hi - d_lo < n and z_hi - z_lo < n, j
    assert executed > 0


def test_plan_rejects_bad_geometry():
    w = S.small_workload(n=64)
    g = w.geometry_kwargs()
    with pytest.raises(apic.ApicError) as e:
        apic.Plan({**g, "n": 96})
    assert e.value.code == apic.APIC_EUNSUPPORTED
    bad = np.array(w.k_bf)
    bad[0] = (14, 0)  # NA-matched LED outside the pupil (r = 12.3)
    with pytest.raises(apic.ApicError) as e:
        apic.Plan({**g, "k_bf": bad})
    assert e.value.code == apic.APIC_EINVAL
    far = np.array(w.k_df)
    far[0] = (30, 0)  # shifted support would wrap the 64-grid
    with pytest.raises(apic.ApicError) as e:
        apic.Plan({**g, "k_df": far})
    assert e.value.code == apic.APIC_EUNSUPPORTED


def test_calls_reject_bad_arguments_without_a_gpu():
    w = S.small_workload(n=64)
    plan = apic.Plan(w.geometry_kwargs())
    lib = plan.lib
    descs = apic.tile_descs(2, 16, 64, 128 * 128)
    need = plan.workspace_bytes(descs)
    assert need > 0
    fake = ctypes.c_void_p(1 << 20)
    # workspace too small
    rc = lib.apic_reconstruct_tiles(plan.handle, 2, descs, fake, None, fake, fake, fake, fake,
                                    need - 1, None)
    assert rc == apic.APIC_EINVAL
    # null outputs
    rc = lib.apic_reconstruct_tiles(plan.handle, 2, descs, fake, None, None, fake, fake, fake,
                                    need, None)
    assert rc == apic.APIC_EINVAL
    # bad geometry index in a descriptor
    descs[1].geom = 3
    rc = lib.apic_workspace_bytes(plan.handle, 2, descs, ctypes.byref(ctypes.c_size_t()))
    assert rc == apic.APIC_EINVAL
    # corrupted plan handle
    junk = (ctypes.c_uint32 * 64)()
    rc = lib.apic_workspace_bytes(ctypes.cast(junk, ctypes.c_void_p), 0, None,
                                  ctypes.byref(ctypes.c_size_t()))
    assert rc == apic.APIC_EPLAN
    # empty batch is a no-op
    assert lib.apic_reconstruct_tiles(plan.handle, 0, None, None, None, None, None, None, None, 0,
                                      None) == apic.APIC_OK
    # background statistic: image offsets must allow 16-byte loads
    descs = apic.tile_descs(2, 16, 64, 0)
    descs[1].image_offset += 2
    rc = lib.apic_background_stat(plan.handle, 2, descs, fake, fake, fake, need, None)
    assert rc == apic.APIC_EINVAL
    # pixel-domain pupil solve: bad tolerance / iteration cap; too many pupil pixels
    rc = lib.apic_estimate_pupil_pixel(plan.handle, 2, descs, fake, 0.0, 100, fake, fake, None,
                                       fake, fake, need, None)
    assert rc == apic.APIC_EINVAL
    rc = lib.apic_estimate_pupil_pixel(plan.handle, 2, descs, fake, 1e-10, 0, fake, fake, None,
                                       fake, fake, need, None)
    assert rc == apic.APIC_EINVAL
    # a plan of several geometry classes is refused (one class per call); a
    # valid plan's pupil (r < N/4, N <= 512) stays under the 65536-pixel limit
    two = apic.Plan([S.small_workload(n=64).geometry_kwargs(),
                     S.small_workload(n=128).geometry_kwargs()])
    rc = lib.apic_estimate_pupil_pixel(two.handle, 2, descs, fake, 1e-10, 100, fake, fake,
                                       None, fake, fake, need, None)
    assert rc == apic.APIC_EUNSUPPORTED
    # assembly: layout arguments, bad handle, ramp width >= 1
    pos = (ctypes.c_int32 * 4)(0, 0, 0, 8)
    h = ctypes.c_void_p()
    assert lib.apic_assembly_create(2, 16, pos, 1, 0, 32, ctypes.byref(h)) == apic.APIC_EINVAL
    assert lib.apic_assembly_create(0, 16, pos, 1, 32, 32, ctypes.byref(h)) == apic.APIC_EINVAL
    assert lib.apic_assembly_create(2, 16, None, 1, 32, 32, ctypes.byref(h)) == apic.APIC_EINVAL
    rc = lib.apic_blend(ctypes.cast(junk, ctypes.c_void_p), fake, None, 4.0, fake, None)
    assert rc == apic.APIC_EINVAL
    # streamer: chunk >= 1, 2..4 buffers, geometry in range, null output handle
    h = ctypes.c_void_p()
    for geom, chunk, nbuf in ((0, 0, 3), (0, 4, 1), (0, 4, 5), (1, 4, 3), (-1, 4, 3)):
        rc = lib.apic_streamer_create(plan.handle, geom, chunk, nbuf, ctypes.byref(h))
        assert rc == apic.APIC_EINVAL and not h.value
    assert lib.apic_streamer_create(plan.handle, 0, 4, 3, None) == apic.APIC_EINVAL
    rc = lib.apic_streamer_run(ctypes.cast(junk, ctypes.c_void_p), 1, None, None, None, None,
                               0.05, 1e6, 1.0, 0.0, None, None, None)
    assert rc == apic.APIC_EINVAL


def test_workspace_grows_with_tiles_and_mixed_classes():
    a = S.small_workload(n=64)
    b = S.small_workload(n=128, n_bf=12, n_df=24, na_df=(0.30, 0.38))
    plan = apic.Plan([a.geometry_kwargs(), b.geometry_kwargs()])
    one = apic.tile_descs(1, 16, 64, 0)
    two = apic.tile_descs(2, 16, 64, 0)
    assert plan.workspace_bytes(two) > plan.workspace_bytes(one)
    mixed = apic.tile_descs(2, 16, 64, 0)
    mixed[1].geom = 1
    assert plan.workspace_bytes(mixed) > plan.workspace_bytes(two)


def test_surrogate_checkpoint_round_trip(tmp_path):
    """Parameters, input normalisation and Adam state survive save / load
    (host tensors; no GPU needed)."""
    theta = apic.init_mlp_params(3)
    sur = apic.Surrogate(theta, np.arange(34.0), np.ones(34) * 2.0, device="cpu")
    sur.m += 0.25
    sur.v += 0.5
    sur.t = 123
    path = tmp_path / "sur.npz"
    sur.save(path)
    back = apic.Surrogate.load(path, device="cpu")
    assert np.array_equal(back.theta.numpy(), theta)
    assert np.array_equal(back.mean.numpy(), np.arange(34.0, dtype=np.float32))
    assert np.array_equal(back.m.numpy(), sur.m.numpy()) and np.array_equal(back.v.numpy(), sur.v.numpy())
    assert back.t == 123


def test_surrogate_positions_are_checked_on_the_host():
    """The surrogate kernels read positions row t for every tile t: a buffer of
    the wrong shape or off the GPU is refused before any call."""
    import torch
    from paper_2407_20469_amd import apic
    with pytest.raises(ValueError):
        apic._positions(torch.zeros((3, 2)), 4, None)
    with pytest.raises(ValueError):
        apic._positions(torch.zeros((4, 3)), 4, None)
    with pytest.raises(ValueError):
        apic._positions(np.zeros((4, 2), np.float32), 4, None)
    with pytest.raises(ValueError):  # right shape, host memory
        apic._positions(torch.zeros((4, 2)), 4, None)
