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


def band_rel_l2(field, ref, geom):
    """Relative L2 errors of the output spectrum over the darkfield band (the
    frequencies the darkfield extension adds: known at the end, outside every
    NA-matched support) and over the brightfield band, comparing fft2 of the
    two fN x fN fields at the embedded N x N frequencies.  The whole-field norm
    is dominated by the low frequencies; the darkfield band carries little
    energy and is checked on its own."""
    from oracle.grid import k_grid, circ
    n = geom.n
    nf = np.asarray(field).shape[-1]
    ky, kx = k_grid(n)
    bf = np.zeros((n, n), bool)
    for k in geom.k_bf:
        bf |= circ(ky + k[1], kx + k[0], geom.r)
    df = np.asarray(ref["known"]) & ~bf
    yy, xx = np.mod(ky, nf), np.mod(kx, nf)
    fg = np.fft.fft2(np.asarray(field, dtype=np.complex128))[yy, xx]
    fo = np.fft.fft2(np.asarray(ref["field"], dtype=np.complex128))[yy, xx]
    return rel_l2(fg[df], fo[df]), rel_l2(fg[bf], fo[bf])
