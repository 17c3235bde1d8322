"""The pupil solve at large aberrations and its seeds, on the GPU through the
C ABI, against the FP64 oracle.

* Coarse-to-fine continuation (the plan default): on tiles of the 1024-tile
  benchmark workload (256 px, 16 NA-matched LEDs, quadratic field model up to
  1.5 rad, Poisson 1e4), the GPU's coefficients match the oracle's within the
  contract bar (1e-3 rad); both recover the truth, which the single pass of
  Eq. 10 (pupil_bands = 0) misses by tenths of a radian or more because beta
  wraps.
* A caller's seed together with the surrogate in its replacing role: the
  fallback rule judges both candidates on the sums re-wrapped about the
  caller's seed, as increments over it; every tile's decision matches the
  oracle's rule evaluated the same way.
* A caller's seed with the surrogate seeding the solve is rejected.

Tolerances: Zernike 1e-3 rad (contract); decisions identical away from the
thresholds (1e-3 relative), as in the surrogate tests.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import apic_synth as S
import apic_synth.surrogate_set as SS
from apic_synth.batch import synth_batch
from oracle import fallback as FB
from paper_2407_20469_amd import apic

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TILES = [0, 31, 200, 527, 613, 1000]


def _log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def grid_tiles():
    w = S.grid_batch()
    imgs = synth_batch(w, torch.device(DEV), tiles=TILES)[:, :w.n_bf].contiguous()
    return w, imgs


def test_continuation_matches_oracle_and_truth_at_1p5_rad(grid_tiles):
    w, imgs = grid_tiles
    g = w.geometry_kwargs()
    g_bf = {**g, "k_df": np.zeros((0, 2), np.int64)}
    _log(f"continuation on {len(TILES)} benchmark tiles")
    z, diag, _, st = apic.estimate_pupil(apic.Plan(g_bf), imgs)
    z1, _, _, _ = apic.estimate_pupil(apic.Plan({**g_bf, "pupil_bands": 0}), imgs)
    z, z1 = z.cpu().numpy(), z1.cpu().numpy()
    host = imgs.cpu().numpy().astype(np.float64)
    og = oracle.Geometry(**g_bf)
    for t, tile in enumerate(TILES):
        spectra, _ = oracle.pipeline.kk_stack(host[t], og)
        ref = oracle.estimate_pupil(spectra, og.k_bf, og.r)
        truth = w.coeffs[tile]
        d_or = np.abs(z[t] - ref["c"]).max()
        e_gpu = np.linalg.norm(z[t, 3:] - truth[3:])
        e_one = np.linalg.norm(z1[t, 3:] - truth[3:])
        _log(f"  tile {tile}: max|c| {np.abs(truth).max():.2f}, |dc| vs oracle {d_or:.2e}, "
             f"error vs truth {e_gpu:.4f} (single pass {e_one:.3f}), R {diag[t, 0]:.4f}")
        assert d_or < 1e-3, tile
        assert e_gpu < 0.02, tile
        assert e_one > 0.2, tile


def test_caller_seed_with_surrogate_decisions_match_oracle():
    """A batch given both a seed and the surrogate.  The final pass is
    re-wrapped about the caller's seed, so both candidates are judged as
    increments over it."""
    dev = torch.device(DEV)
    geom = SS.geometry()
    plan = apic.Plan(geom)
    rng = np.random.default_rng(41)
    T = 24
    uv = rng.uniform(-1, 1, (T, 2))
    imgs, c_true = SS.make_tiles(uv, rng.uniform(size=T) < 0.3, seed=12, device=dev)
    seed = (c_true + rng.normal(0, 0.05, c_true.shape) * (np.arange(15) >= 3)).astype(np.float32)
    seed_dev = torch.tensor(seed, device=dev)
    pos = torch.tensor(uv, dtype=torch.float32, device=dev)
    sur = apic.Surrogate(apic.init_mlp_params(23), np.zeros(34), np.ones(34), device=DEV)
    _, _, feat, _ = apic.estimate_pupil(plan, imgs)
    x = torch.cat([pos, feat], dim=1)
    zs = sur.forward(x).cpu().numpy().astype(np.float64)
    g = oracle.Geometry(**geom)
    host = imgs.cpu().numpy().astype(np.float64)
    ref = []
    for t in range(T):
        spectra, _ = oracle.pipeline.kk_stack(host[t], g)
        out = oracle.estimate_pupil(spectra, g.k_bf, g.r, seed=seed[t].astype(np.float64))
        ref.append((out["sums"], float(np.linalg.cond(out["sums"]["A"])), out["c"]))
    rhos = [FB.choose(s, c[3:], zs[t], k, 0.0, 1e30, 1e30, c0=seed[t, 3:])[1]
            for t, (s, k, c) in enumerate(ref)]
    rho_max = float(np.median(rhos))
    _log(f"caller seed + surrogate: oracle rho {min(rhos):.3g} .. {max(rhos):.3g}")
    n, n_img = geom["n"], imgs.shape[1]
    nf = 2 * n
    descs = apic.tile_descs(T, n_img, n, nf * nf)
    batch = apic.Batch(plan, descs)
    batch.set_surrogate(sur, pos, rho_max=rho_max, kappa_max=1e6, resid_max=1.0)
    field = torch.empty(T * nf * nf, dtype=torch.complex64, device=dev)
    zb = torch.empty((T, 15), dtype=torch.float32, device=dev)
    sb = torch.empty((T,), dtype=torch.int32, device=dev)
    batch.reconstruct(imgs.reshape(-1), field, zb, sb, apic.Workspace(), seed=seed_dev)
    torch.cuda.synchronize()
    zb, sb = zb.cpu().numpy(), sb.cpu().numpy()
    compared, outcomes = 0, set()
    for t, (sums, kappa, c_cf) in enumerate(ref):
        use_sur, rho, r_cf = FB.choose(sums, c_cf[3:], zs[t], kappa, rho_max, 1e6, 1.0,
                                       c0=seed[t, 3:])
        if abs(rho - rho_max) < 1e-3 * rho_max or abs(r_cf - 1.0) < 1e-3:
            continue
        compared += 1
        outcomes.add(use_sur)
        assert bool(sb[t] & apic.TILE_SURROGATE_USED) == use_sur, t
        assert bool(sb[t] & apic.TILE_FALLBACK_USED) == (not use_sur), t
        assert sb[t] & apic.TILE_SEEDED
        want = zs[t] if use_sur else c_cf[3:]
        assert np.abs(zb[t, 3:] - want).max() < 1e-3, t
    _log(f"  {compared} of {T} tiles compared, outcomes {sorted(outcomes)}")
    assert compared >= T - 2 and outcomes == {True, False}
    # the surrogate seeding the solve does not take a caller's seed as well
    sur.seeds_solve = True
    batch.set_surrogate(sur, pos)
    with pytest.raises(apic.ApicError) as e:
        batch.reconstruct(imgs.reshape(-1), field, torch.empty((T, 15), device=dev),
                          torch.empty((T,), dtype=torch.int32, device=dev), apic.Workspace(),
                          seed=seed_dev)
    assert e.value.code == apic.APIC_EINVAL
    batch.close()
