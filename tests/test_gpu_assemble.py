"""Patch assembly on the GPU (Sec. 2.5 overlap blending at known positions)
against the FP64 oracle.

Case 1: a 3 x 4 grid of 64 px tiles cut with 16 px overlaps from one random
complex field, each tile given its own constant phase and independent noise,
plus two tiles that overlap only each other.  Bars: phases within 1e-5 rad of
the oracle's eigenvector phases (FP64 correlations on both sides; the host
power iteration stops at a 1e-14 change); canvas within 1e-5 relative (FP32
weighted sums) of the oracle's blend with the oracle's phases.
Case 2: four overlapping windows of a larger object reconstructed by the GPU
(64 px tiles, 2x output): GPU assembly = oracle assembly of the same fields,
and the alignment shrinks the disagreement between overlapping tiles.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import apic_synth as S
from oracle import assemble as oa
from paper_2407_20469_amd import apic

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _log(msg):
    print(f"[gpu-test] {msg}", flush=True)


def test_assembly_matches_oracle():
    rng = np.random.default_rng(3)
    n, stride = 64, 48
    H, W = 2 * stride + n + 80, 3 * stride + n
    field = S.object_smooth(rng, 256)[:H, :W]
    pos = [(i * stride, j * stride) for i in range(3) for j in range(4)]
    pos += [(H - n, 0), (H - n, 40)]   # a pair that overlaps only each other
    pos = np.array(pos)
    tiles = np.stack([field[y:y + n, x:x + n] for y, x in pos])
    ph = rng.uniform(-np.pi, np.pi, len(pos))
    noise = 0.01 * (rng.standard_normal(tiles.shape) + 1j * rng.standard_normal(tiles.shape))
    tiles = (tiles + noise) * np.exp(1j * ph)[:, None, None]
    t32 = tiles.astype(np.complex64)
    _log(f"{len(pos)} tiles on a {H} x {W} canvas")
    canvas, theta = apic.assemble(torch.tensor(t32, device=DEV), pos, (H, W), 16.0)
    t64 = t32.astype(np.complex128)
    th_ref = oa.synchronise_phases(oa.overlap_matrix(t64, pos))
    d = np.angle(np.exp(1j * (theta - th_ref)))
    _log(f"max |dtheta| {np.abs(d).max():.2e}")
    assert np.abs(d).max() < 1e-5
    ref = oa.blend(t64, pos, th_ref, (H, W), 16.0)
    got = canvas.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _log(f"canvas max rel err {err:.2e}")
    assert err < 1e-5
    covered = np.zeros((H, W), bool)
    for y, x in pos:
        covered[y:y + n, x:x + n] = True
    assert np.all(got[~covered] == 0)


def test_reconstructed_windows_assemble():
    n, stride = 64, 48
    big = S.object_smooth(np.random.default_rng([9, 0, 0]), 256)
    w = S.small_workload(n=n, n_tiles=4, seed_id=51)
    pos_in = [(0, 0), (0, stride), (stride, 0), (stride, stride)]
    k_all = list(w.k_bf) + list(w.k_df)
    imgs = np.stack([oracle.forward_images(big[y:y + n, x:x + n], k_all, w.coeffs[t], w.r)
                     for t, (y, x) in enumerate(pos_in)]).astype(np.float32)
    plan = apic.Plan(w.geometry_kwargs())
    field, z, st = apic.reconstruct(plan, torch.tensor(imgs, device=DEV))
    nf = n * w.upsample
    pos = np.array(pos_in) * w.upsample
    H = W = stride * w.upsample + nf
    canvas, theta = apic.assemble(field, pos, (H, W), 32.0, min_overlap=8)
    f64 = field.cpu().numpy().astype(np.complex128)
    th_ref = oa.synchronise_phases(oa.overlap_matrix(f64, pos, min_overlap=8))
    d = np.angle(np.exp(1j * (theta - th_ref)))
    ref = oa.blend(f64, pos, th_ref, (H, W), 32.0)
    err = np.abs(canvas.cpu().numpy() - ref).max() / np.abs(ref).max()
    _log(f"reconstructed windows: max |dtheta| {np.abs(d).max():.2e}, canvas rel err {err:.2e}")
    assert np.abs(d).max() < 1e-5 and err < 1e-5

    def mismatch(th):
        tot = 0.0
        for t in range(4):
            for u in range(t + 1, 4):
                y0, x0 = np.maximum(pos[t], pos[u])
                y1, x1 = np.minimum(pos[t], pos[u]) + nf
                a = f64[t][y0 - pos[t][0]:y1 - pos[t][0], x0 - pos[t][1]:x1 - pos[t][1]]
                b = f64[u][y0 - pos[u][0]:y1 - pos[u][0], x0 - pos[u][1]:x1 - pos[u][1]]
                tot += np.sum(np.abs(a * np.exp(-1j * th[t]) - b * np.exp(-1j * th[u])) ** 2)
        return tot
    before, after = mismatch(np.zeros(4)), mismatch(theta.astype(np.float64))
    _log(f"overlap mismatch {before:.3e} -> {after:.3e}")
    assert after <= before
