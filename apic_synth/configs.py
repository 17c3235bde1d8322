"""Workload recipes (geometry, objects, true pupils, noise) for the synthetic
benchmarks.  Common optics: lambda = 0.52 um, objective NA 0.25, sample pixel
0.4 um, so the pupil radius is r = 0.19231 N bins.
"""

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .leds import led_rings
from .objects import object_background, object_smooth

OPTICS = {"dx_um": 0.4, "wavelength_um": 0.52, "na_obj": 0.25}


@dataclass
class Workload:
    """A set of tiles sharing one geometry class."""
    name: str
    n: int
    k_bf: List
    k_df: List
    upsample: int = 2
    n_tiles: int = 1
    photons: Optional[float] = None      # Poisson scale per unit clear intensity
    seed_id: int = 0
    obj_fn: Callable = object_smooth       # (rng, n) -> complex object
    coeffs: Optional[np.ndarray] = None  # (n_tiles, 15) true Noll coefficients
    positions: Optional[np.ndarray] = None  # (n_tiles, 2) normalised (u, v)
    dx_um: float = OPTICS["dx_um"]
    wavelength_um: float = OPTICS["wavelength_um"]
    na_obj: float = OPTICS["na_obj"]
    extra: dict = field(default_factory=dict)

    @property
    def r(self):
        return self.na_obj * self.n * self.dx_um / self.wavelength_um

    @property
    def n_bf(self):
        return len(self.k_bf)

    @property
    def n_df(self):
        return len(self.k_df)

    @property
    def n_img(self):
        return len(self.k_bf) + len(self.k_df)

    def object(self, tile):
        rng = np.random.default_rng([self.seed_id, 0, tile])
        background = self.extra.get("background")
        if background is not None and background[tile]:
            return object_background(rng, self.n)
        return self.obj_fn(rng, self.n)

    def geometry_kwargs(self):
        return {"n": self.n, "dx_um": self.dx_um, "wavelength_um": self.wavelength_um,
                "na_obj": self.na_obj, "k_bf": np.asarray(self.k_bf, np.int64),
                "k_df": np.asarray(self.k_df, np.int64), "upsample": self.upsample}


def pupil_random(seed=(0, 2, 0)):
    """c_j ~ N(0, 0.5^2) for Noll j in {4, 5, 6, 7, 8, 11}, others 0."""
    rng = np.random.default_rng(list(seed))
    c = np.zeros(15)
    for j in (4, 5, 6, 7, 8, 11):
        c[j - 1] = rng.normal(0.0, 0.5)
    return c


def single_tile():
    """One 128 x 128 tile, 8 NA-matched LEDs at NA 0.25 and 8 darkfield at 0.32,
    noise-free, smooth object, 2x output."""
    n = 128
    leds_bf = led_rings(n, [(0.25, 8, 0.0, True)])
    leds_df = led_rings(n, [(0.32, 8, 0.0, False)])
    return Workload("single128", n, leds_bf, leds_df, upsample=2, n_tiles=1, photons=None,
                    seed_id=0, coeffs=pupil_random()[None, :], positions=np.zeros((1, 2)))


def field_model_quadratic(u, v, max_abs=1.5):
    """Noll c_4..c_15 quadratic in the field position (u, v), rescaled so that the
    largest |c| over the given positions equals ``max_abs`` rad."""
    rng = np.random.default_rng([2407, 20469])
    a = rng.normal(0.0, 1.0, size=(12, 6))
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    basis = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], axis=-1)
    c = np.zeros(u.shape + (15,))
    c[..., 3:15] = basis @ a.T
    scale = max_abs / np.abs(c).max()
    return c * scale, a * scale


def grid_batch(n_tiles=1024, photons=1e4, n=256):
    """1024 tiles of 256^2 on a 32 x 32 field grid; 16 NA-matched LEDs at 0.25,
    16 darkfield at 0.30 and 16 at 0.38 (half-step azimuth offset); Poisson noise."""
    leds_bf = led_rings(n, [(0.25, 16, 0.0, True)])
    leds_df = led_rings(n, [(0.30, 16, 0.0, False), (0.38, 16, 0.5, False)])
    g = np.arange(1024)
    u = (g % 32 - 15.5) / 15.5
    v = (g // 32 - 15.5) / 15.5
    c_all, _ = field_model_quadratic(u, v)
    pos = np.stack([u, v], axis=1)
    return Workload("grid256", n, leds_bf, leds_df, upsample=2, n_tiles=n_tiles, photons=photons,
                    seed_id=1, coeffs=c_all[:n_tiles], positions=pos[:n_tiles])


def small_workload(n=64, n_bf=8, n_df=8, na_df=(0.32,), n_tiles=2, photons=None, seed_id=7):
    """A small geometry (default 64^2) for quick parity checks; same optics."""
    leds_bf = led_rings(n, [(0.25, n_bf, 0.0, True)])
    rings = [(na, n_df // len(na_df), 0.5 * (m % 2), False) for m, na in enumerate(na_df)]
    leds_df = led_rings(n, rings)
    coeffs = np.stack([pupil_random((seed_id, 2, t)) * 0.5 for t in range(n_tiles)])
    return Workload(f"small{n}", n, leds_bf, leds_df, upsample=2, n_tiles=n_tiles,
                    photons=photons, seed_id=seed_id, coeffs=coeffs,
                    positions=np.zeros((n_tiles, 2)))


def uneven_classes():
    """The nine geometry classes of the uneven batch: N in {128, 256, 512} x
    n_bf in {8, 12, 16}, n_df = 2 n_bf on rings at NA 0.30 and 0.38."""
    out = []
    for n in (128, 256, 512):
        for n_bf in (8, 12, 16):
            leds_bf = led_rings(n, [(0.25, n_bf, 0.0, True)])
            leds_df = led_rings(n, [(0.30, n_bf, 0.0, False), (0.38, n_bf, 0.5, False)])
            out.append({"n": n, "n_bf": n_bf, "k_bf": leds_bf, "k_df": leds_df})
    return out


def uneven_tiles(n_tiles=4096, seed=2, background_fraction=0.4, random_positions=False):
    """Per-tile (size, n_bf, background, position) of the uneven batch: sizes
    128/256/512 in the ratio 4:3:1, n_bf uniform in {8, 12, 16}, 40%
    background tiles (``background_fraction``), on a square field grid
    (64 x 64 for 4096 tiles) or, with ``random_positions``, at positions
    uniform over [-1, 1]^2 (``default_rng([2, 3, seed])``)."""
    rng = np.random.default_rng([2, 2, seed])
    sizes = np.array([128] * (n_tiles // 2) + [256] * (3 * n_tiles // 8)
                     + [512] * (n_tiles - n_tiles // 2 - 3 * n_tiles // 8))
    rng.shuffle(sizes)
    nbf = rng.choice([8, 12, 16], size=n_tiles)
    bg = np.zeros(n_tiles, dtype=bool)
    bg[rng.choice(n_tiles, size=int(round(background_fraction * n_tiles)), replace=False)] = True
    if random_positions:
        uv = np.random.default_rng([2, 3, seed]).uniform(-1.0, 1.0, (n_tiles, 2))
        u, v = uv[:, 0], uv[:, 1]
    else:
        g = np.arange(n_tiles)
        side = int(round(np.sqrt(n_tiles)))
        u = (g % side - (side - 1) / 2) / ((side - 1) / 2)
        v = (g // side - (side - 1) / 2) / ((side - 1) / 2)
    return {"n": sizes, "n_bf": nbf, "background": bg, "u": u, "v": v}


def field_model_on_grid(u, v, side=64):
    """The quadratic field model with the scale fitted on a side x side grid
    of [-1, 1]^2 (max |c| = 1.5 rad there), evaluated at positions (u, v)."""
    g = np.arange(side * side)
    _, a = field_model_quadratic((g % side - (side - 1) / 2) / ((side - 1) / 2),
                                 (g // side - (side - 1) / 2) / ((side - 1) / 2))
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    c = np.zeros(u.shape + (15,))
    c[..., 3:15] = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], axis=-1) @ a.T
    return c


def uneven_batch(n_tiles=4096, photons=1e4, seed=2, background_fraction=0.4,
                 random_positions=False, darkfield=True, seed_base=20):
    """The uneven batch as one Workload per geometry class (in the order of
    ``uneven_classes``), each with the batch-wide indices of its tiles in
    ``extra["tiles"]`` and its background flags in ``extra["background"]``.
    True pupils follow the quadratic field model at each tile's position,
    scaled on the batch's own grid (random positions: on the 64 x 64 grid of
    the 4096-tile batch).  ``darkfield=False``
    drops the darkfield images (a training set for the surrogate, whose inputs
    and labels come from the NA-matched images only); ``seed_base`` gives the
    classes' object and noise seeds (seed_base + class)."""
    classes = uneven_classes()
    tiles = uneven_tiles(n_tiles, seed, background_fraction, random_positions)
    if random_positions:
        c_all = field_model_on_grid(tiles["u"], tiles["v"])
    else:
        c_all, _ = field_model_quadratic(tiles["u"], tiles["v"])
    out = []
    for ci, g in enumerate(classes):
        sel = np.nonzero((tiles["n"] == g["n"]) & (tiles["n_bf"] == g["n_bf"]))[0]
        if len(sel) == 0:
            continue
        out.append(Workload(f"uneven-{g['n']}-{g['n_bf']}", g["n"], g["k_bf"],
                            g["k_df"] if darkfield else [],
                            upsample=2, n_tiles=len(sel), photons=photons,
                            seed_id=seed_base + ci, coeffs=c_all[sel],
                            positions=np.stack([tiles["u"][sel], tiles["v"][sel]], axis=1),
                            extra={"tiles": sel, "background": tiles["background"][sel],
                                   "class": ci}))
    return out


def surrogate_train_batch(n_tiles=16384):
    """Training set of the learned-surrogate workload: content tiles of the
    uneven recipe (no background), NA-matched images only, at uniform random
    field positions; objects and noise from their own seeds (classes 40..48),
    so the set is disjoint from the evaluation set."""
    return uneven_batch(n_tiles, seed=5, background_fraction=0.0, random_positions=True,
                        darkfield=False, seed_base=40)


def surrogate_eval_batch(n_tiles=4096):
    """Evaluation set of the learned-surrogate workload: the uneven recipe with
    70% background tiles and all darkfield images, on the 64 x 64 grid
    (classes 60..68)."""
    return uneven_batch(n_tiles, seed=6, background_fraction=0.7, seed_base=60)
