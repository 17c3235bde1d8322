"""Large synthetic batches: objects drawn per tile with NumPy (seeded
default_rng([seed_id, 0, tile])), images formed with torch on the target device
in float64, Poisson noise drawn there per chunk of 32 tiles (torch generator
seeded with seed_id * 1000003 + first tile of the chunk), cast to float32.

The objects of the next chunk are drawn on host threads while the device forms
the current chunk's images; each object depends only on its own seed, so the
result does not depend on the thread count."""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from .imaging import form_images, add_poisson

CHUNK = 32
_POOL = None


def _pool():
    global _POOL
    if _POOL is None:
        _POOL = ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)))
    return _POOL


def synth_batch(w, device, tiles=None, chunk=CHUNK, log=None):
    """float32 tensor (T, n_bf + n_df, N, N) on ``device`` for workload ``w``.

    ``tiles`` selects a subset (list of tile indices); noise chunks follow the
    full-batch chunking so a tile gets the same noise whatever subset is drawn.
    """
    tiles = list(range(w.n_tiles)) if tiles is None else list(tiles)
    k_all = [tuple(k) for k in w.k_bf] + [tuple(k) for k in w.k_df]
    out = torch.empty((len(tiles), len(k_all), w.n, w.n), dtype=torch.float32, device=device)
    by_chunk = {}
    for pos, t in enumerate(tiles):
        by_chunk.setdefault(t // chunk, []).append((pos, t))
    items = sorted(by_chunk.items())

    def draw(i):
        first = items[i][0] * chunk
        return [_pool().submit(w.object, t) for t in range(first, min(w.n_tiles, first + chunk))]

    pending = draw(0) if items else None
    for done, (cidx, members) in enumerate(items):
        first = cidx * chunk
        full = list(range(first, min(w.n_tiles, first + chunk)))
        futs = pending
        pending = draw(done + 1) if done + 1 < len(items) else None
        objs = np.stack([f.result() for f in futs])
        imgs = form_images(objs, w.coeffs[full], k_all, w.r, device=device, dtype=torch.float64)
        if w.photons:
            imgs = add_poisson(imgs, w.photons, seed=w.seed_id * 1000003 + first, device=device)
        for pos, t in members:
            out[pos] = imgs[t - first].to(torch.float32)
        if log and (done % 8 == 0):
            log(f"synth: chunk {done + 1}/{len(by_chunk)}")
    return out
