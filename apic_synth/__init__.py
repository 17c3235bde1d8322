"""Seeded synthetic inputs for the per-tile APIC reconstruction.

This module is the only code shared by the FP64 oracle (``oracle/``), the tests,
and the GPU product path's benchmark.  It holds no step of the reconstruction
method: it draws illumination lattices, objects, true pupil coefficients, tile
grids and noise, and it forms intensity images from them (Eq. 1-2 of the paper,
the microscope's side, implemented here a third time with torch so that large
batches can be synthesised on the GPU; it is pinned against the oracle's own
forward model by the tests).

Every random draw uses ``numpy.random.default_rng([seed_id, stream, tile])`` with
streams 0 = object, 1 = noise, 2 = per-tile draws; the field-dependence model
shared by the multi-tile workloads uses ``default_rng([2407, 20469])``.
"""

from .leds import led_ring, led_rings
from .objects import (gaussian_smooth_periodic, minmax, object_smooth, object_background,
                      object_blobs)
from .configs import (OPTICS, Workload, single_tile, grid_batch, uneven_batch, uneven_classes, uneven_tiles,
                      field_model_quadratic, field_model_on_grid, pupil_random, small_workload,
                      surrogate_train_batch, surrogate_eval_batch)
from .imaging import form_images, add_poisson

__all__ = [
    "led_ring", "led_rings", "gaussian_smooth_periodic", "minmax", "object_smooth",
    "object_background", "object_blobs", "OPTICS", "Workload", "single_tile", "grid_batch",
    "uneven_batch", "uneven_classes", "uneven_tiles", "field_model_quadratic", "field_model_on_grid",
    "pupil_random", "small_workload", "surrogate_train_batch", "surrogate_eval_batch",
    "form_images", "add_poisson",
]
