"""ctypes binding of libapic.so (the C ABI in include/apic.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of the library.  torch tensors provide device memory and streams.
Importing this module does not need a GPU; calling an entry point does.  If
the library is not built, loading raises instead of falling back to anything.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapic.so")

APIC_OK, APIC_EINVAL, APIC_EUNSUPPORTED, APIC_EHIP, APIC_ENOMEM, APIC_EPLAN = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "APIC_OK", -1: "APIC_EINVAL", -2: "APIC_EUNSUPPORTED", -3: "APIC_EHIP",
                -4: "APIC_ENOMEM", -5: "APIC_EPLAN"}

TILE_SKIP_DARKFIELD = 0x1  # descriptor flag
TILE_NONFINITE_INPUT = 0x001
TILE_LOG_FLOOR = 0x002
TILE_PUPIL_ILLCOND = 0x004
TILE_PUPIL_CHOL_FAIL = 0x008
TILE_DF_CHOL_FAIL = 0x010
TILE_DF_SKIPPED = 0x020
TILE_SEEDED = 0x040
TILE_NONFINITE_OUT = 0x080
TILE_SURROGATE_USED = 0x100
TILE_FALLBACK_USED = 0x200
TILE_BACKGROUND = 0x400
TILE_PIXEL_NOT_CONVERGED = 0x800
MLP_PARAMS, MLP_INPUTS, MLP_OUTPUTS = 26896, 34, 12
TILE_SKIP_DARKFIELD = 0x1

EXPORTS = ["apic_plan_create", "apic_plan_destroy", "apic_plan_upload", "apic_workspace_bytes",
           "apic_plan_query", "apic_reconstruct_tiles", "apic_reconstruct_tiles_static",
           "apic_estimate_pupil", "apic_kk_spectra",
           "apic_stitch_brightfield", "apic_extend_darkfield", "apic_upsample_field", "apic_fft2",
           "apic_profile", "apic_profile_read", "apic_calib_fma64", "apic_calib_mfma64", "apic_calib_copy",
           "apic_mlp_forward", "apic_mlp_train", "apic_mlp_grad", "apic_bf16_gemm",
           "apic_estimate_pupil_sur", "apic_reconstruct_tiles_sur", "apic_batch_create",
           "apic_batch_destroy", "apic_batch_workspace_bytes", "apic_batch_reconstruct",
           "apic_batch_capture", "apic_batch_launch", "apic_batch_classes", "apic_batch_set_chunk", "apic_batch_set_surrogate",
           "apic_batch_autotune", "apic_batch_fit", "apic_batch_set_fft", "apic_batch_fft_panel",
           "apic_background_stat",
           "apic_estimate_pupil_pixel", "apic_assembly_create", "apic_assembly_destroy",
           "apic_assemble_phases", "apic_blend", "apic_rgb_combine",
           "apic_streamer_create", "apic_streamer_destroy", "apic_streamer_device_bytes",
           "apic_streamer_run", "apic_version"]

PROF_GROUPS = ["kk", "pupil", "stitch", "df_fft", "df_rhs", "gram", "chol", "out"]


class ApicError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} returned {STATUS_NAMES.get(code, code)}")
        self.code = code


class Geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("upsample", ctypes.c_int32),
                ("dx_um", ctypes.c_double), ("wavelength_um", ctypes.c_double),
                ("na_obj", ctypes.c_double), ("n_bf", ctypes.c_int32), ("n_df", ctypes.c_int32),
                ("k_bf", ctypes.POINTER(ctypes.c_int32)), ("k_df", ctypes.POINTER(ctypes.c_int32)),
                ("ridge_pupil", ctypes.c_double), ("ridge_darkfield", ctypes.c_double),
                ("log_floor_rel", ctypes.c_double), ("pupil_bands", ctypes.c_int32)]


class MlpModel(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p), ("in_mean", ctypes.c_void_p),
                ("in_std", ctypes.c_void_p), ("seeds_solve", ctypes.c_int32)]


class TileDesc(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("image_offset", ctypes.c_int64), ("field_offset", ctypes.c_int64),
                ("pos_x", ctypes.c_float), ("pos_y", ctypes.c_float)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libapic.so (raises if it has not been built).

    torch is imported first: it carries its own HIP runtime, and the library
    must bind to that same runtime (loading a second one first leaves torch
    without devices)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"libapic.so not found at {path}: run "
                           "`python -m paper_2407_20469_amd.build` (hipcc, gfx950) first")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.apic_plan_create.argtypes = [ctypes.POINTER(Geometry), i32, ctypes.POINTER(P)]
    lib.apic_plan_destroy.argtypes = [P]
    lib.apic_plan_upload.argtypes = [P]
    lib.apic_workspace_bytes.argtypes = [P, i32, ctypes.POINTER(TileDesc), ctypes.POINTER(sz)]
    lib.apic_plan_query.argtypes = [P, i32, i32, i32, ctypes.POINTER(i32), i64,
                                    ctypes.POINTER(i64)]
    lib.apic_reconstruct_tiles.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, P, P, P, sz,
                                           P]
    lib.apic_reconstruct_tiles_static.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, P, P,
                                                  P]
    lib.apic_estimate_pupil.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, P, P, P, P, sz,
                                        P]
    lib.apic_kk_spectra.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, P, sz, P]
    lib.apic_stitch_brightfield.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, P, P, sz, P]
    lib.apic_extend_darkfield.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, P, P, sz, P]
    lib.apic_upsample_field.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, sz, P]
    lib.apic_fft2.argtypes = [i32, i32, i32, i32, P, P, P]
    lib.apic_mlp_forward.argtypes = [ctypes.POINTER(MlpModel), i32, P, P, P]
    lib.apic_mlp_train.argtypes = [P, P, P, P, P, P, i32, P, P, P, i32, i32, i32, ctypes.c_float,
                                   P, P]
    lib.apic_mlp_grad.argtypes = [P, P, P, P, i32, P, P, P, i32, P, P]
    lib.apic_bf16_gemm.argtypes = [i32, i32, i32, P, P, P, P]
    f32 = ctypes.c_float
    lib.apic_estimate_pupil_sur.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P,
                                            ctypes.POINTER(MlpModel), f32, f32, f32, P, P, P, P, P,
                                            P, sz, P]
    lib.apic_reconstruct_tiles_sur.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P,
                                               ctypes.POINTER(MlpModel), f32, f32, f32, P, P, P, P,
                                               sz, P]
    lib.apic_batch_create.argtypes = [P, i32, ctypes.POINTER(TileDesc), ctypes.POINTER(P)]
    lib.apic_batch_destroy.argtypes = [P]
    lib.apic_batch_workspace_bytes.argtypes = [P, ctypes.POINTER(sz)]
    lib.apic_batch_reconstruct.argtypes = [P, P, P, P, P, P, P, sz, P]
    lib.apic_batch_capture.argtypes = [P, P, P, P, P, P, P, sz, P]
    lib.apic_batch_launch.argtypes = [P, P]
    lib.apic_batch_classes.argtypes = [P, ctypes.POINTER(i32), P, P, P, P, P]
    lib.apic_batch_set_chunk.argtypes = [P, i32, i32, i32]
    lib.apic_batch_set_surrogate.argtypes = [P, P, P, f32, f32, f32]
    lib.apic_batch_autotune.argtypes = [P, i32, P, P, P, P, P, sz, P, ctypes.c_double, P]
    lib.apic_batch_fit.argtypes = [P, sz]
    lib.apic_batch_set_fft.argtypes = [P, i32, i32]
    lib.apic_batch_fft_panel.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.apic_background_stat.argtypes = [P, i32, ctypes.POINTER(TileDesc), P, P, P, sz, P]
    lib.apic_rgb_combine.argtypes = [i32, i32, P, P, P, P, P, P, P, sz, P]
    lib.apic_assembly_create.argtypes = [i32, i32, P, i32, i32, i32, ctypes.POINTER(P)]
    lib.apic_assembly_destroy.argtypes = [P]
    lib.apic_assemble_phases.argtypes = [P, P, P, P]
    lib.apic_blend.argtypes = [P, P, P, ctypes.c_float, P, P]
    lib.apic_estimate_pupil_pixel.argtypes = [P, i32, ctypes.POINTER(TileDesc), P,
                                              ctypes.c_double, i32, P, P, P, P, P, sz, P]
    lib.apic_streamer_create.argtypes = [P, i32, i32, i32, ctypes.POINTER(P)]
    lib.apic_streamer_destroy.argtypes = [P]
    lib.apic_streamer_device_bytes.argtypes = [P, ctypes.POINTER(sz)]
    lib.apic_streamer_run.argtypes = [P, i32, P, P, P, ctypes.POINTER(MlpModel), f32, f32, f32,
                                      f32, P, P, P]
    lib.apic_calib_fma64.argtypes = [P, i32, i32, P]
    lib.apic_calib_mfma64.argtypes = [P, i32, i32, P]
    lib.apic_calib_copy.argtypes = [P, P, i64, P]
    lib.apic_profile.argtypes = [i32]
    lib.apic_profile_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_double)]
    for name in EXPORTS:
        getattr(lib, name).restype = ctypes.c_char_p if name == "apic_version" else ctypes.c_int
    _lib = lib
    return lib


def _check(fn, code):
    if code != APIC_OK:
        raise ApicError(fn, code)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A plan over one or more geometry classes (dicts with keys n, upsample,
    dx_um, wavelength_um, na_obj, k_bf, k_df and optional ridges/log floor)."""

    def __init__(self, geometries):
        self.lib = load_library()
        if isinstance(geometries, dict):
            geometries = [geometries]
        self.geoms = [dict(g) for g in geometries]
        self._keep = []
        arr = (Geometry * len(self.geoms))()
        for g, c in zip(self.geoms, arr):
            kbf = np.ascontiguousarray(np.asarray(g["k_bf"], dtype=np.int32).reshape(-1, 2))
            kdf = np.ascontiguousarray(np.asarray(g.get("k_df", np.zeros((0, 2))),
                                                  dtype=np.int32).reshape(-1, 2))
            self._keep += [kbf, kdf]
            c.n = int(g["n"])
            c.upsample = int(g.get("upsample", 2))
            c.dx_um = float(g["dx_um"])
            c.wavelength_um = float(g["wavelength_um"])
            c.na_obj = float(g["na_obj"])
            c.n_bf = kbf.shape[0]
            c.n_df = kdf.shape[0]
            c.k_bf = kbf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            c.k_df = kdf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            c.ridge_pupil = float(g.get("ridge_pupil", 1e-9))
            c.ridge_darkfield = float(g.get("ridge_darkfield", 1e-4))
            c.log_floor_rel = float(g.get("log_floor_rel", 1e-6))
            c.pupil_bands = int(g.get("pupil_bands", 1))
            g["n_bf"], g["n_df"] = int(c.n_bf), int(c.n_df)
        self.handle = ctypes.c_void_p()
        _check("apic_plan_create", self.lib.apic_plan_create(arr, len(self.geoms),
                                                             ctypes.byref(self.handle)))

    def close(self):
        if self.handle:
            self.lib.apic_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload(self):
        _check("apic_plan_upload", self.lib.apic_plan_upload(self.handle))

    def query(self, what, geom=0, j=0):
        n = ctypes.c_int64()
        _check("apic_plan_query", self.lib.apic_plan_query(self.handle, geom, what, j, None, 0,
                                                           ctypes.byref(n)))
        out = np.zeros(max(1, n.value), dtype=np.int32)
        _check("apic_plan_query", self.lib.apic_plan_query(
            self.handle, geom, what, j, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            out.size, ctypes.byref(n)))
        return out[:n.value]

    def sizes(self, geom=0):
        v = self.query(5, geom)
        return dict(zip(["n_pairs", "n_rows", "nu_max", "m_max", "ne_max", "n_active", "gram_block",
                         "gram_chunk", "n_pix"], v.tolist()))

    def workspace_bytes(self, descs):
        b = ctypes.c_size_t()
        _check("apic_workspace_bytes", self.lib.apic_workspace_bytes(
            self.handle, len(descs), descs, ctypes.byref(b)))
        return b.value


def tile_descs(n_tiles, n_img, n, out_elems, geom=0, flags=0, positions=None):
    """Descriptors of a contiguous batch: tile t's images at t * n_img * N^2 and
    its output at t * out_elems."""
    arr = (TileDesc * n_tiles)()
    for t in range(n_tiles):
        arr[t].geom = geom
        arr[t].flags = flags
        arr[t].image_offset = t * n_img * n * n
        arr[t].field_offset = t * out_elems
        if positions is not None:
            arr[t].pos_x, arr[t].pos_y = float(positions[t][0]), float(positions[t][1])
    return arr


class Workspace:
    """Caller-owned device scratch (a torch uint8 tensor, 256-B aligned)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        import torch
        if self.buf is None or self.buf.numel() < nbytes + 256 or self.buf.device != device:
            self.buf = None
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        return ctypes.c_void_p((base + 255) & ~255), nbytes


def mixed_descs(plan, geom_ids, flags=None):
    """Descriptors for tiles of several geometry classes packed back to back in
    one flat image buffer and one flat field buffer, in the given order.
    Returns (descs, image elements, field elements)."""
    geom_ids = np.asarray(geom_ids, dtype=np.int64)
    arr = (TileDesc * len(geom_ids))()
    io = fo = 0
    for t, gi in enumerate(geom_ids):
        g = plan.geoms[int(gi)]
        n, nf = g["n"], g["n"] * g.get("upsample", 2)
        arr[t].geom = int(gi)
        arr[t].flags = 0 if flags is None else int(flags[t])
        arr[t].image_offset = io
        arr[t].field_offset = fo
        io += (g["n_bf"] + g["n_df"]) * n * n
        fo += nf * nf
    return arr, io, fo


class Batch:
    """A prepared batch (apic_batch_*): tile descriptors resident on the device,
    the geometry classes run concurrently on side streams, and one call can be
    captured into a graph and replayed.  ``descs`` as for the plain calls;
    images are a flat float32 buffer and fields a flat complex64 buffer that
    the descriptors index."""

    def __init__(self, plan, descs):
        self.plan, self.lib, self.descs = plan, plan.lib, descs
        self.n_tiles = len(descs)
        self.handle = ctypes.c_void_p()
        _check("apic_batch_create", self.lib.apic_batch_create(
            plan.handle, self.n_tiles, descs, ctypes.byref(self.handle)))
        self._refresh()
        self._bound = None
        need_img = need_fld = 0
        for d in descs:
            g = plan.geoms[d.geom]
            n, nf = g["n"], g["n"] * g.get("upsample", 2)
            need_img = max(need_img, d.image_offset + (g["n_bf"] + g["n_df"]) * n * n)
            need_fld = max(need_fld, d.field_offset + nf * nf)
        self.image_elems, self.field_elems = need_img, need_fld

    def _refresh(self):
        b = ctypes.c_size_t()
        _check("apic_batch_workspace_bytes",
               self.lib.apic_batch_workspace_bytes(self.handle, ctypes.byref(b)))
        self.workspace_bytes = b.value

    def classes(self):
        """[{geom, n_tiles, chunk, lanes, tile_bytes, fft_variant, fft_panel_columns}] in the
        order the batch runs them."""
        n = ctypes.c_int32(0)
        _check("apic_batch_classes", self.lib.apic_batch_classes(self.handle, ctypes.byref(n),
                                                                 None, None, None, None, None))
        cap = n.value
        g, t, c, ln = (np.zeros(max(cap, 1), np.int32) for _ in range(4))
        b = np.zeros(max(cap, 1), np.int64)
        _check("apic_batch_classes", self.lib.apic_batch_classes(
            self.handle, ctypes.byref(n), g.ctypes.data_as(ctypes.c_void_p),
            t.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p),
            ln.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p)))
        out = []
        for i in range(cap):
            var, cols = ctypes.c_int32(0), ctypes.c_int32(0)
            _check("apic_batch_fft_panel", self.lib.apic_batch_fft_panel(
                self.handle, i, ctypes.byref(var), ctypes.byref(cols)))
            out.append({"geom": int(g[i]), "n_tiles": int(t[i]), "chunk": int(c[i]),
                        "lanes": int(ln[i]), "tile_bytes": int(b[i]), "fft_variant": var.value,
                        "fft_panel_columns": cols.value})
        return out

    def set_fft(self, cls, variant):
        """Panel variant of class ``cls``'s FFT column passes (apic_batch_set_fft)."""
        _check("apic_batch_set_fft", self.lib.apic_batch_set_fft(self.handle, cls, variant))
        self._bound = None

    def set_chunk(self, cls, tiles, lanes=1):
        _check("apic_batch_set_chunk", self.lib.apic_batch_set_chunk(self.handle, cls, tiles,
                                                                     lanes))
        self._refresh()
        self._bound = None

    def set_surrogate(self, sur, positions, rho_max=0.05, kappa_max=1e6, resid_max=1.0):
        """Run the surrogate and its fallback rule in every later call of this
        batch (apic_batch_set_surrogate); ``sur=None`` switches it off.
        ``positions`` is a float32 (T, 2) device tensor in batch order.  The
        batch borrows the model's and the positions' device memory, so both
        are kept referenced here."""
        import torch
        if sur is None:
            _check("apic_batch_set_surrogate", self.lib.apic_batch_set_surrogate(
                self.handle, None, None, 0.0, 0.0, 0.0))
            self._sur = None
        else:
            pos = _positions(positions, self.n_tiles, images_device=None)
            mdl = sur.model()
            _check("apic_batch_set_surrogate", self.lib.apic_batch_set_surrogate(
                self.handle, ctypes.byref(mdl), _ptr(pos), float(rho_max), float(kappa_max),
                float(resid_max)))
            self._sur = (sur, mdl, pos)
        self._bound = None

    def autotune(self, images, field, zernike, status, workspace_ptr, workspace_bytes,
                 slack=0.05, stream=None, log=None):
        """Pick each class's chunk and lanes by timing (see apic_batch_autotune),
        one class per call so that `log` (optional) reports progress, then fit
        the classes into the budget.  The workspace is a raw 256-B aligned
        device pointer and its size.  Returns the best ms per tile per class."""
        classes = self.classes()
        ms = np.zeros(max(len(classes), 1), np.float64)
        self._args(images, field, zernike, status, None, None)
        for ci, c in enumerate(classes):
            _check("apic_batch_autotune", self.lib.apic_batch_autotune(
                self.handle, ci, _ptr(images), _ptr(zernike), _ptr(field), _ptr(status),
                workspace_ptr, workspace_bytes, _stream(stream), float(slack),
                ms.ctypes.data_as(ctypes.c_void_p)))
            if log:
                t = self.classes()[ci]
                log(f"autotune class {ci} (geometry {t['geom']}, {t['n_tiles']} tiles): chunk "
                    f"{t['chunk']}, lanes {t['lanes']}, {ms[ci]:.3f} ms per tile")
        _check("apic_batch_fit", self.lib.apic_batch_fit(self.handle, workspace_bytes))
        self._refresh()
        self._bound = None
        return ms[:len(classes)]

    def fit(self, workspace_bytes):
        """Halve the largest classes' chunks until the classes' workspace blocks
        together fit ``workspace_bytes`` (apic_batch_fit), without timing runs."""
        _check("apic_batch_fit", self.lib.apic_batch_fit(self.handle, int(workspace_bytes)))
        self._refresh()
        self._bound = None

    def close(self):
        if self.handle:
            self.lib.apic_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _args(self, images, field, zernike, status, workspace, seed):
        import torch
        if images.dtype != torch.float32 or not images.is_contiguous() or \
                images.numel() < self.image_elems:
            raise ValueError("images: contiguous float32 with room for every descriptor")
        if field.dtype != torch.complex64 or not field.is_contiguous() or \
                field.numel() < self.field_elems:
            raise ValueError("field: contiguous complex64 with room for every descriptor")
        if zernike.numel() < 15 * self.n_tiles or status.numel() < self.n_tiles:
            raise ValueError("zernike (T, 15) and status (T,) buffers too small")
        if seed is not None and (seed.dtype != torch.float32 or seed.numel() < 15 * self.n_tiles):
            raise ValueError("seed must be float32 (T, 15)")
        if workspace is None:
            return None
        wp, wb = workspace.get(self.workspace_bytes, images.device)
        return [_ptr(images), _ptr(seed), _ptr(zernike), _ptr(field), _ptr(status), wp, wb]

    def reconstruct(self, images, field, zernike, status, workspace, seed=None, stream=None):
        """Enqueue the whole method for the batch on ``stream``; no host sync."""
        _check("apic_batch_reconstruct", self.lib.apic_batch_reconstruct(
            self.handle, *self._args(images, field, zernike, status, workspace, seed),
            _stream(stream)))

    def capture(self, images, field, zernike, status, workspace, stream, seed=None):
        """Record one reconstruct call on ``stream`` (a non-default torch stream)
        into the batch's graph; the buffers stay bound to it for launch()."""
        if stream is None:
            raise ValueError("capture needs an explicit non-default stream")
        args = self._args(images, field, zernike, status, workspace, seed)
        _check("apic_batch_capture", self.lib.apic_batch_capture(self.handle, *args,
                                                                 _stream(stream)))
        self._bound = (images, field, zernike, status, workspace, seed)

    def launch(self, stream=None):
        if self._bound is None:
            raise RuntimeError("launch before capture")
        _check("apic_batch_launch", self.lib.apic_batch_launch(self.handle, _stream(stream)))


def _positions(positions, n_tiles, images_device):
    """Surrogate positions as a contiguous float32 (T, 2) device tensor; the
    kernels read row t for every tile t, so the shape is checked here."""
    import torch
    if not isinstance(positions, torch.Tensor) or positions.shape != (n_tiles, 2):
        raise ValueError(f"positions must be a ({n_tiles}, 2) tensor")
    if positions.device.type != "cuda" or (images_device is not None and
                                           positions.device != images_device):
        raise ValueError("positions must live on the images' GPU")
    return positions.to(torch.float32).contiguous()


def _batch_args(plan, images, geom=0):
    g = plan.geoms[geom]
    n, n_img = g["n"], g["n_bf"] + g["n_df"]
    if images.dim() != 4 or images.shape[1:] != (n_img, n, n):
        raise ValueError(f"images must be (T, {n_img}, {n}, {n}), got {tuple(images.shape)}")
    if not images.is_cuda or images.dtype.__str__() != "torch.float32" or not images.is_contiguous():
        raise ValueError("images must be a contiguous float32 CUDA tensor")
    return g, n, n_img, images.shape[0]


def reconstruct(plan, images, seed=None, workspace=None, stream=None):
    """Whole method on a contiguous single-geometry batch (T, n_img, N, N).
    Returns (field complex64 (T, fN, fN), zernike (T, 15), status (T,))."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    nf = n * g.get("upsample", 2)
    dev = images.device
    field = torch.empty((T, nf, nf), dtype=torch.complex64, device=dev)
    zern = torch.empty((T, 15), dtype=torch.float32, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, nf * nf)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    if seed is not None:
        seed = seed.contiguous().to(torch.float32)
    _check("apic_reconstruct_tiles", plan.lib.apic_reconstruct_tiles(
        plan.handle, T, descs, _ptr(images), _ptr(seed), _ptr(zern), _ptr(field), _ptr(status),
        wp, wb, _stream(stream)))
    return field, zern, status


def estimate_pupil(plan, images, seed=None, workspace=None, stream=None):
    """Eq. 4-10 on a batch.  Returns (zernike (T,15), diag (T,4), features (T,32), status)."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    dev = images.device
    zern = torch.empty((T, 15), dtype=torch.float32, device=dev)
    diag = torch.empty((T, 4), dtype=torch.float32, device=dev)
    feat = torch.empty((T, 32), dtype=torch.float32, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, 0)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    if seed is not None:
        seed = seed.contiguous().to(torch.float32)
    _check("apic_estimate_pupil", plan.lib.apic_estimate_pupil(
        plan.handle, T, descs, _ptr(images), _ptr(seed), _ptr(zern), _ptr(diag), _ptr(feat),
        _ptr(status), wp, wb, _stream(stream)))
    return zern, diag, feat, status


def estimate_pupil_pixel(plan, images, tol=1e-10, max_iter=1000, workspace=None, stream=None):
    """Eq. 10 with one unknown per pupil pixel.  Returns (phi (T, N, N) float32
    in FFT order, zernike summary (T, 15), iterations (T,), status (T,))."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    dev = images.device
    phi = torch.empty((T, n, n), dtype=torch.float32, device=dev)
    zern = torch.empty((T, 15), dtype=torch.float32, device=dev)
    iters = torch.empty((T,), dtype=torch.int32, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, 0)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    _check("apic_estimate_pupil_pixel", plan.lib.apic_estimate_pupil_pixel(
        plan.handle, T, descs, _ptr(images), float(tol), int(max_iter), _ptr(phi), _ptr(zern),
        _ptr(iters), _ptr(status), wp, wb, _stream(stream)))
    return phi, zern, iters, status


def rgb_combine(field_r, field_g, field_b, gains=None, stream=None):
    """Colour image (T, 3, nf, nf) float32 of three channel fields (complex64
    CUDA (T, nf, nf)): g_c |F_c|, grey-world gains unless given.  Returns
    (image, gains)."""
    import torch
    fs = [f.contiguous() for f in (field_r, field_g, field_b)]
    if any(f.dtype != torch.complex64 or not f.is_cuda or f.shape != fs[0].shape for f in fs):
        raise ValueError("three complex64 CUDA fields of one shape (T, nf, nf)")
    T, nf = fs[0].shape[0], fs[0].shape[-1]
    out = torch.empty((T, 3, nf, nf), dtype=torch.float32, device=fs[0].device)
    g_in = None if gains is None else np.ascontiguousarray(np.asarray(gains, np.float32))
    g_out = np.zeros(3, np.float32)
    ws = torch.empty(3 * 1024 * 8 + 256, dtype=torch.uint8, device=fs[0].device)
    wp = (ws.data_ptr() + 255) & ~255
    _check("apic_rgb_combine", load_library().apic_rgb_combine(
        T, nf, _ptr(fs[0]), _ptr(fs[1]), _ptr(fs[2]),
        None if g_in is None else g_in.ctypes.data_as(ctypes.c_void_p), _ptr(out),
        g_out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(wp), 3 * 1024 * 8,
        _stream(stream)))
    return out, g_out


class Assembly:
    """Tiles of side n at integer canvas positions (T, 2) (row, column) on a
    canvas of ``canvas_shape``: overlapping pairs and per-block tile lists
    prepared once on the device (see apic_assembly_create)."""

    def __init__(self, n, positions, canvas_shape, min_overlap=1):
        self.lib = load_library()
        self.pos = np.ascontiguousarray(np.asarray(positions, np.int32).reshape(-1, 2))
        self.T, self.n = self.pos.shape[0], int(n)
        self.shape = (int(canvas_shape[0]), int(canvas_shape[1]))
        h = ctypes.c_void_p()
        _check("apic_assembly_create", self.lib.apic_assembly_create(
            self.T, self.n, self.pos.ctypes.data_as(ctypes.c_void_p), int(min_overlap),
            self.shape[0], self.shape[1], ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.apic_assembly_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fields(self, fields):
        import torch
        f = fields.contiguous()
        if (f.dtype != torch.complex64 or not f.is_cuda or f.numel() != self.T * self.n ** 2):
            raise ValueError(f"fields must be complex64 CUDA ({self.T}, {self.n}, {self.n})")
        return f

    def phases(self, fields, stream=None):
        """Constant phase of each tile (NumPy float32 (T,))."""
        f = self._fields(fields)
        theta = np.zeros(self.T, np.float32)
        _check("apic_assemble_phases", self.lib.apic_assemble_phases(
            self.handle, _ptr(f), theta.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return theta

    def blend(self, fields, theta, ramp_width, out=None, stream=None):
        """Blend onto a complex64 canvas; theta a float32 CUDA tensor (T,) or None."""
        import torch
        f = self._fields(fields)
        canvas = out if out is not None else torch.empty(self.shape, dtype=torch.complex64,
                                                         device=f.device)
        th = None if theta is None else theta.contiguous().to(torch.float32)
        _check("apic_blend", self.lib.apic_blend(
            self.handle, _ptr(f), _ptr(th), float(ramp_width), _ptr(canvas), _stream(stream)))
        return canvas


def assemble(fields, positions, canvas_shape, ramp_width, min_overlap=1, align_phases=True,
             stream=None):
    """Phase-align (unless ``align_phases`` is False) and blend tiles (complex64
    CUDA (T, n, n)) at integer canvas positions.  Returns (canvas, theta)."""
    import torch
    a = Assembly(fields.shape[-1], positions, canvas_shape, min_overlap)
    theta = a.phases(fields, stream) if align_phases else np.zeros(a.T, np.float32)
    canvas = a.blend(fields, torch.tensor(theta, device=fields.device), ramp_width,
                     stream=stream)
    a.close()
    return canvas, theta


def background_stat(plan, images, workspace=None, stream=None):
    """Background statistic of each tile (float32 tensor (T,)): mean over the
    NA-matched images of var(I) / mean(I)^2."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    out = torch.empty((T,), dtype=torch.float32, device=images.device)
    descs = tile_descs(T, n_img, n, 0)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), images.device)
    _check("apic_background_stat", plan.lib.apic_background_stat(
        plan.handle, T, descs, _ptr(images), _ptr(out), wp, wb, _stream(stream)))
    return out


class Streamer:
    """Slide stream: tiles of geometry ``geom`` whose image stacks are in host
    memory, reconstructed in chunks of ``chunk`` tiles through ``n_buffers``
    device staging buffers, each on its own stream (see apic_streamer_run)."""

    def __init__(self, plan, geom=0, chunk=8, n_buffers=3):
        self.plan = plan
        self.lib = plan.lib
        self.geom = plan.geoms[geom]
        h = ctypes.c_void_p()
        _check("apic_streamer_create", self.lib.apic_streamer_create(
            plan.handle, geom, chunk, n_buffers, ctypes.byref(h)))
        self.handle = h

    @property
    def device_bytes(self):
        b = ctypes.c_size_t()
        _check("apic_streamer_device_bytes",
               self.lib.apic_streamer_device_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.apic_streamer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, host_images, host_fields, positions=None, sur=None, rho_max=0.05,
            kappa_max=1e6, resid_max=1.0, bg_threshold=0.0):
        """host_images / host_fields: sequences of CPU tensors (pinned for
        asynchronous copies), one per tile; the fields are complex64 (fN, fN).
        Returns (zernike (T, 15), status (T,), background statistic (T,)) as
        NumPy arrays."""
        T = len(host_images)
        if len(host_fields) != T:
            raise ValueError("one field buffer per tile")
        n, nf = self.geom["n"], self.geom["n"] * self.geom.get("upsample", 2)
        n_img = self.geom["n_bf"] + self.geom["n_df"]
        for x in host_images:
            if x.is_cuda or x.numel() != n_img * n * n or not x.is_contiguous():
                raise ValueError("each image stack is a contiguous host tensor (n_img, N, N)")
        for f in host_fields:
            if f.is_cuda or f.numel() * f.element_size() != 8 * nf * nf or not f.is_contiguous():
                raise ValueError("each field is a contiguous host complex64 (fN, fN)")
        imgs = (ctypes.c_void_p * T)(*[x.data_ptr() for x in host_images])
        flds = (ctypes.c_void_p * T)(*[f.data_ptr() for f in host_fields])
        z = np.zeros((T, 15), np.float32)
        st = np.zeros(T, np.uint32)
        bg = np.zeros(T, np.float32)
        pos = None
        mdl = None
        if sur is not None:
            pos = np.ascontiguousarray(np.asarray(positions, np.float32).reshape(T, 2))
            mdl = sur.model()
        _check("apic_streamer_run", self.lib.apic_streamer_run(
            self.handle, T, imgs, flds,
            None if pos is None else pos.ctypes.data_as(ctypes.c_void_p),
            None if mdl is None else ctypes.byref(mdl), float(rho_max), float(kappa_max),
            float(resid_max), float(bg_threshold), z.ctypes.data_as(ctypes.c_void_p),
            st.ctypes.data_as(ctypes.c_void_p), bg.ctypes.data_as(ctypes.c_void_p)))
        return z, st, bg


def kk_spectra(plan, images, workspace=None, stream=None):
    """KK spectra (T, n_bf, N, N) complex64."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    dev = images.device
    out = torch.empty((T, g["n_bf"], n, n), dtype=torch.complex64, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, 0)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    _check("apic_kk_spectra", plan.lib.apic_kk_spectra(
        plan.handle, T, descs, _ptr(images), _ptr(out), _ptr(status), wp, wb, _stream(stream)))
    return out, status


def stitch_brightfield(plan, images, zernike, workspace=None, stream=None):
    """Corrected, stitched brightfield spectra (T, N, N) complex64."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    dev = images.device
    out = torch.empty((T, n, n), dtype=torch.complex64, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, n * n)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    z = zernike.contiguous().to(torch.float32)
    _check("apic_stitch_brightfield", plan.lib.apic_stitch_brightfield(
        plan.handle, T, descs, _ptr(images), _ptr(z), _ptr(out), _ptr(status), wp, wb,
        _stream(stream)))
    return out, status


def extend_darkfield(plan, images, zernike, spectrum, workspace=None, stream=None):
    """Eq. 11-13 in place on a copy of `spectrum` (T, N, N) complex64."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    dev = images.device
    spec = spectrum.contiguous().clone()
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, n * n)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    z = zernike.contiguous().to(torch.float32)
    _check("apic_extend_darkfield", plan.lib.apic_extend_darkfield(
        plan.handle, T, descs, _ptr(images), _ptr(z), _ptr(spec), _ptr(status), wp, wb,
        _stream(stream)))
    return spec, status


def upsample_field(plan, spectrum, workspace=None, stream=None):
    """fN x fN fields from (T, N, N) complex64 spectra."""
    import torch
    g = plan.geoms[0]
    n, nf = g["n"], g["n"] * g.get("upsample", 2)
    T = spectrum.shape[0]
    spec = spectrum.contiguous()
    out = torch.empty((T, nf, nf), dtype=torch.complex64, device=spec.device)
    descs = tile_descs(T, g["n_bf"] + g["n_df"], n, nf * nf)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), spec.device)
    _check("apic_upsample_field", plan.lib.apic_upsample_field(
        plan.handle, T, descs, _ptr(spec), _ptr(out), wp, wb, _stream(stream)))
    return out


def profile(enable):
    """Start (True) or stop (False) recording kernel-group timings."""
    _check("apic_profile", load_library().apic_profile(int(bool(enable))))


def profile_read():
    """{group: (total_ms, launches, total_work)} of the recorded launches."""
    lib = load_library()
    out = {}
    for gid, name in enumerate(PROF_GROUPS):
        ms, n, work = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check("apic_profile_read", lib.apic_profile_read(gid, ctypes.byref(ms), ctypes.byref(n),
                                                          ctypes.byref(work)))
        out[name] = (ms.value, n.value, work.value)
    return out


def fft2(x, inverse=False, stream=None):
    """Unnormalised batched 2D FFT of (B, L, L) complex64/complex128 CUDA tensors."""
    import torch
    lib = load_library()
    x = x.contiguous()
    prec = 1 if x.dtype == torch.complex128 else 0
    out = torch.empty_like(x)
    _check("apic_fft2", lib.apic_fft2(x.shape[-1], x.numel() // (x.shape[-1] ** 2), int(inverse),
                                      prec, _ptr(x), _ptr(out), _stream(stream)))
    return out


# ---------------------------------------------------------------- surrogate
class Surrogate:
    """Device-resident surrogate model: FP32 parameters, input normalisation and
    Adam state (torch tensors on one device)."""

    def __init__(self, theta, in_mean, in_std, device="cuda"):
        import torch
        self.theta = torch.as_tensor(np.asarray(theta, np.float32), device=device).contiguous()
        self.mean = torch.as_tensor(np.asarray(in_mean, np.float32), device=device).contiguous()
        self.std = torch.as_tensor(np.asarray(in_std, np.float32), device=device).contiguous()
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.t = 0
        self.seeds_solve = False    # True: the prediction seeds the re-wrapped pupil solve

    def model(self):
        return MlpModel(self.theta.data_ptr(), self.mean.data_ptr(), self.std.data_ptr(),
                        int(bool(self.seeds_solve)))

    def save(self, path):
        """Checkpoint: parameters, input normalisation and Adam state (.npz)."""
        np.savez(path, theta=self.theta.cpu().numpy(), in_mean=self.mean.cpu().numpy(),
                 in_std=self.std.cpu().numpy(), adam_m=self.m.cpu().numpy(),
                 adam_v=self.v.cpu().numpy(), adam_t=np.int64(self.t))

    @classmethod
    def load(cls, path, device="cuda"):
        """Resume from a checkpoint written by save()."""
        import torch
        with np.load(path, allow_pickle=False) as f:
            sur = cls(f["theta"], f["in_mean"], f["in_std"], device=device)
            sur.m = torch.as_tensor(f["adam_m"], device=device).contiguous()
            sur.v = torch.as_tensor(f["adam_v"], device=device).contiguous()
            sur.t = int(f["adam_t"])
        return sur

    def forward(self, inputs, stream=None):
        import torch
        x = inputs.contiguous().to(torch.float32)
        out = torch.empty((x.shape[0], MLP_OUTPUTS), dtype=torch.float32, device=x.device)
        mdl = self.model()
        _check("apic_mlp_forward", load_library().apic_mlp_forward(
            ctypes.byref(mdl), x.shape[0], _ptr(x), _ptr(out), _stream(stream)))
        return out

    def train(self, inputs, targets, order, batch, lr=1e-3, stream=None):
        """len(order) // batch Adam steps; returns the per-step losses."""
        import torch
        x = inputs.contiguous().to(torch.float32)
        y = targets.contiguous().to(torch.float32)
        order = torch.as_tensor(order, dtype=torch.int32, device=x.device).contiguous()
        steps = order.numel() // batch
        loss = torch.empty(steps, dtype=torch.float32, device=x.device)
        _check("apic_mlp_train", load_library().apic_mlp_train(
            _ptr(self.theta), _ptr(self.m), _ptr(self.v), _ptr(self.grad), _ptr(self.mean),
            _ptr(self.std), x.shape[0], _ptr(x), _ptr(y), _ptr(order), steps, batch, self.t,
            float(lr), _ptr(loss), _stream(stream)))
        self.t += steps
        return loss

    def gradient(self, inputs, targets, order, stream=None):
        """Loss and gradient over the samples listed in order (no update)."""
        import torch
        x = inputs.contiguous().to(torch.float32)
        y = targets.contiguous().to(torch.float32)
        order = torch.as_tensor(order, dtype=torch.int32, device=x.device).contiguous()
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        grad = torch.empty_like(self.theta)
        _check("apic_mlp_grad", load_library().apic_mlp_grad(
            _ptr(self.theta), _ptr(grad), _ptr(self.mean), _ptr(self.std), x.shape[0], _ptr(x),
            _ptr(y), _ptr(order), order.numel(), _ptr(loss), _stream(stream)))
        return loss, grad


def init_mlp_params(seed=0):
    """He-style uniform initial parameters (FP32 flat vector); padded input
    columns of W1 and padded output rows of W3 are zero."""
    rng = np.random.default_rng(seed)
    w1 = np.zeros((128, 64))
    w1[:, :34] = rng.uniform(-1, 1, (128, 34)) * np.sqrt(6.0 / 34)
    w2 = rng.uniform(-1, 1, (128, 128)) * np.sqrt(6.0 / 128)
    w3 = np.zeros((16, 128))
    w3[:12] = rng.uniform(-1, 1, (12, 128)) * np.sqrt(3.0 / 128)
    parts = [w1, np.zeros(128), w2, np.zeros(128), w3, np.zeros(16)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def bf16_gemm(a_bits, b_bits, stream=None):
    """c = a b for bfloat16 bit patterns (int16/uint16 tensors), FP32 result."""
    import torch
    m, k = a_bits.shape
    n = b_bits.shape[1]
    c = torch.empty((m, n), dtype=torch.float32, device=a_bits.device)
    _check("apic_bf16_gemm", load_library().apic_bf16_gemm(
        m, n, k, _ptr(a_bits.contiguous()), _ptr(b_bits.contiguous()), _ptr(c), _stream(stream)))
    return c


def estimate_pupil_sur(plan, images, positions, sur, rho_max=0.05, kappa_max=1e6,
                       resid_max=1.0, workspace=None, stream=None):
    """Pupil with the surrogate and fallback rule.  Returns (chosen, closed form,
    surrogate, diag, status), Zernike arrays (T, 15)."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    dev = images.device
    z, zcf, zsur = (torch.empty((T, 15), dtype=torch.float32, device=dev) for _ in range(3))
    diag = torch.empty((T, 4), dtype=torch.float32, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, 0)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    pos = _positions(positions, T, images.device)
    mdl = sur.model()
    _check("apic_estimate_pupil_sur", plan.lib.apic_estimate_pupil_sur(
        plan.handle, T, descs, _ptr(images), _ptr(pos), ctypes.byref(mdl), float(rho_max),
        float(kappa_max), float(resid_max), _ptr(z), _ptr(zcf), _ptr(zsur), _ptr(diag),
        _ptr(status), wp, wb,
        _stream(stream)))
    return z, zcf, zsur, diag, status


def reconstruct_sur(plan, images, positions, sur, rho_max=0.05, kappa_max=1e6, resid_max=1.0,
                    workspace=None, stream=None):
    """Whole method with the surrogate choosing the pupil; (field, zernike, status)."""
    import torch
    g, n, n_img, T = _batch_args(plan, images)
    nf = n * g.get("upsample", 2)
    dev = images.device
    field = torch.empty((T, nf, nf), dtype=torch.complex64, device=dev)
    zern = torch.empty((T, 15), dtype=torch.float32, device=dev)
    status = torch.empty((T,), dtype=torch.int32, device=dev)
    descs = tile_descs(T, n_img, n, nf * nf)
    ws = workspace or Workspace()
    wp, wb = ws.get(plan.workspace_bytes(descs), dev)
    pos = _positions(positions, T, images.device)
    mdl = sur.model()
    _check("apic_reconstruct_tiles_sur", plan.lib.apic_reconstruct_tiles_sur(
        plan.handle, T, descs, _ptr(images), _ptr(pos), ctypes.byref(mdl), float(rho_max),
        float(kappa_max), float(resid_max), _ptr(zern), _ptr(field), _ptr(status), wp, wb,
        _stream(stream)))
    return field, zern, status
