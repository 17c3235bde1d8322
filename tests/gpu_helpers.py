"""Shared helpers of the GPU parity tests: seeded inputs from the oracle's own
forward model (small cases) and relative-error helpers."""

import numpy as np

import oracle
import apic_synth as S


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def workload_images(w, tiles=None, photons=None, seed=11):
    """float32 (T, n_bf + n_df, N, N) from the oracle's forward model."""
    tiles = range(w.n_tiles) if tiles is None else tiles
    k_all = list(w.k_bf) + list(w.k_df)
    out = []
    for t in tiles:
        img = oracle.forward_images(w.object(t), k_all, w.coeffs[t], w.r)
        if photons:
            rng = np.random.default_rng([w.seed_id, 1, t, seed])
            img = rng.poisson(img * photons) / photons
        out.append(img.astype(np.float32))
    return np.stack(out)


def oracle_geometry(w):
    return oracle.Geometry(**w.geometry_kwargs())
