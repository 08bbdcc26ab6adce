"""Python binding of the C ABI in include/dr.h (ctypes, argument marshalling only).

Every function has the name of the C entry point it calls.  Pointers may be
given as integers, torch tensors (device or pinned host; their data_ptr() is
passed) or numpy arrays (host).  Streams may be integers (hipStream_t),
torch streams or None.  Errors raise DRError with the library's message.

The library must be built (``python -m paper_2201_13309_amd.build``); there
is no fallback: importing this module without libdr.so raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdr.so")

DR_OK, DR_PENDING = 0, 1
DR_E_INVAL, DR_E_NOMEM, DR_E_UNSUPPORTED, DR_E_DEVICE, DR_E_BUSY, DR_E_NOTFOUND = (
    -1, -2, -3, -4, -5, -6)
DR_EDGE_LEADING, DR_EDGE_TRAILING, DR_EDGE_BOTH = 0, 1, 2
DR_BATCH_AUTOTUNE, DR_BATCH_GRAPH = 1, 2
DR_PATH_ROWS, DR_PATH_PIXELS = 0, 1
DR_LAYOUT_FULL, DR_LAYOUT_LIST = 0, 1

# names exported by libdr.so, as declared in include/dr.h
ABI_SYMBOLS = (
    "dr_ctx_create", "dr_ctx_destroy", "dr_geometry_init", "dr_geometry_path",
    "dr_geometry_position_margin", "dr_geometry_set_step_weights",
    "dr_geometry_free", "dr_set_tile",
    "dr_autotune", "dr_reconstruct", "dr_reconstruct_f64", "dr_debug_plan", "dr_enable_timing",
    "dr_last_timing", "dr_batch_create", "dr_batch_run", "dr_batch_tile", "dr_batch_free",
    "dr_submit", "dr_poll", "dr_wait", "dr_ctx_stats", "dr_last_error", "dr_pixel_activity",
    "dr_select_top", "dr_list_create", "dr_list_size", "dr_list_pixels", "dr_list_free",
    "dr_reconstruct_list", "dr_reconstruct_list_f64", "dr_reconstruct_noalloc",
)


class DRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class dr_detector(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("u", ctypes.c_double * 3),
                ("v", ctypes.c_double * 3), ("pixel_xyz", ctypes.c_void_p)]


class dr_wire(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_double), ("axis", ctypes.c_double * 3),
                ("n_steps", ctypes.c_int32), ("centers", ctypes.c_void_p),
                ("edge", ctypes.c_int32)]


class dr_depth_grid(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("first_center", ctypes.c_double),
                ("width", ctypes.c_double)]


class dr_tile_config(ctypes.Structure):
    _fields_ = [("pixels_per_lane", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("prefetch", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32)]

    def as_tuple(self):
        return (self.pixels_per_lane, self.waves_per_group, self.prefetch, self.groups_per_cu)


class dr_batch_item(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_void_p), ("images", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("totals", ctypes.c_void_p)]


class dr_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("epochs", ctypes.c_uint64),
                ("tiles_launched", ctypes.c_uint64), ("bytes_h2d", ctypes.c_uint64),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_budget", ctypes.c_size_t)]


_lib = None


def load(path: Optional[str] = None):
    """Load libdr.so; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libdr.so not built ({p}); run python -m paper_2201_13309_amd.build")
    lib = ctypes.CDLL(p)
    vp, i32, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
    P = ctypes.POINTER
    sigs = {
        "dr_ctx_create": [ctypes.c_int, sz, P(vp)],
        "dr_ctx_destroy": [vp],
        "dr_geometry_init": [vp, P(dr_detector), P(dr_wire), P(dr_depth_grid), P(vp)],
        "dr_geometry_path": [vp, P(i32)],
        "dr_geometry_position_margin": [vp, P(ctypes.c_double), P(ctypes.c_double)],
        "dr_geometry_set_step_weights": [vp, vp],
        "dr_geometry_free": [vp],
        "dr_set_tile": [vp, P(dr_tile_config)],
        "dr_autotune": [vp, vp, vp, P(dr_tile_config)],
        "dr_reconstruct": [vp, vp, ctypes.c_int, vp, vp, vp],
        "dr_reconstruct_f64": [vp, vp, vp, vp, vp],
        "dr_reconstruct_noalloc": [vp, vp, vp, vp, vp],
        "dr_debug_plan": [vp, vp, i32, i32, vp, vp],
        "dr_enable_timing": [vp, ctypes.c_int],
        "dr_last_timing": [vp, P(ctypes.c_double), P(ctypes.c_double)],
        "dr_batch_create": [vp, i32, P(dr_batch_item), i32, P(vp)],
        "dr_batch_run": [vp, vp],
        "dr_batch_tile": [vp, P(dr_tile_config)],
        "dr_batch_free": [vp],
        "dr_submit": [vp, vp, vp, ctypes.c_int, vp, vp, P(u64)],
        "dr_poll": [vp, u64],
        "dr_wait": [vp, u64],
        "dr_ctx_stats": [vp, P(dr_stats)],
        "dr_pixel_activity": [vp, vp, vp, vp],
        "dr_select_top": [vp, vp, ctypes.c_int64, P(vp)],
        "dr_list_create": [vp, vp, ctypes.c_int64, ctypes.c_int, P(vp)],
        "dr_list_size": [vp, P(ctypes.c_int64)],
        "dr_list_pixels": [vp, vp],
        "dr_list_free": [vp],
        "dr_reconstruct_list": [vp, vp, i32, ctypes.c_int, vp, vp, vp],
        "dr_reconstruct_list_f64": [vp, vp, i32, vp, vp, vp],
    }
    for name, argt in sigs.items():
        f = getattr(lib, name)
        f.argtypes = argt
        f.restype = ctypes.c_int32
    lib.dr_last_error.argtypes = []
    lib.dr_last_error.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def dr_last_error() -> str:
    return load().dr_last_error().decode(errors="replace")


def _check(rc: int, allow=(DR_OK,)) -> int:
    if rc in allow:
        return rc
    raise DRError(rc, dr_last_error())


def ptr(x) -> Optional[int]:
    """Raw address of a tensor, array or integer (None stays None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    raise TypeError(f"cannot take the address of {type(x)}")


def stream_handle(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


# ------------------------------------------------------------------ context


def dr_ctx_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().dr_ctx_create(device, hbm_budget_bytes, ctypes.byref(h)))
    return h.value


def dr_ctx_destroy(ctx: int) -> None:
    _check(load().dr_ctx_destroy(ctx))


def make_detector(nx, ny, origin, u, v, pixel_xyz: Optional[np.ndarray] = None):
    d = dr_detector()
    d.nx, d.ny = int(nx), int(ny)
    for k in range(3):
        d.origin[k], d.u[k], d.v[k] = float(origin[k]), float(u[k]), float(v[k])
    keep = None
    if pixel_xyz is not None:
        keep = np.ascontiguousarray(pixel_xyz, dtype=np.float64)
        d.pixel_xyz = keep.ctypes.data
    return d, keep


def make_wire(radius, centers, axis=(1.0, 0.0, 0.0), edge: int = DR_EDGE_LEADING):
    c = np.ascontiguousarray(centers, dtype=np.float64)
    w = dr_wire()
    w.radius = float(radius)
    for k in range(3):
        w.axis[k] = float(axis[k])
    w.n_steps = int(c.shape[0])
    w.centers = c.ctypes.data
    w.edge = int(edge)
    return w, c


def dr_geometry_init(ctx: int, detector, wire, grid) -> int:
    """detector / wire / grid: objects with the fields of dr_detector, dr_wire
    and dr_depth_grid (nx, ny, origin, u, v, pixel_xyz; radius, centers, axis;
    n_bins, first_center, width)."""
    d, keep_d = make_detector(detector.nx, detector.ny, detector.origin, detector.u, detector.v,
                              getattr(detector, "pixel_xyz", None))
    w, keep_w = make_wire(wire.radius, wire.centers, getattr(wire, "axis", (1.0, 0.0, 0.0)),
                          getattr(wire, "edge", DR_EDGE_LEADING))
    g = dr_depth_grid()
    g.n_bins, g.first_center, g.width = int(grid.n_bins), float(grid.first_center), float(grid.width)
    h = ctypes.c_void_p()
    rc = load().dr_geometry_init(ctx, ctypes.byref(d), ctypes.byref(w), ctypes.byref(g),
                                 ctypes.byref(h))
    del keep_d, keep_w
    _check(rc)
    weights = getattr(wire, "weights", None)
    if weights is not None:
        try:
            dr_geometry_set_step_weights(h.value, weights)
        except DRError:
            dr_geometry_free(h.value)
            raise
    return h.value


def dr_geometry_set_step_weights(geom: int, weights) -> None:
    """weights: n_steps floats (host), or None to remove them."""
    if weights is None:
        _check(load().dr_geometry_set_step_weights(geom, None))
        return
    w = np.ascontiguousarray(weights, dtype=np.float64)
    _check(load().dr_geometry_set_step_weights(geom, ptr(w)))


def dr_geometry_path(geom: int) -> int:
    """DR_PATH_ROWS or DR_PATH_PIXELS."""
    v = ctypes.c_int32()
    _check(load().dr_geometry_path(geom, ctypes.byref(v)))
    return v.value


def dr_geometry_position_margin(geom: int) -> tuple:
    """(margin, max_error): the margin of the per-pixel path's fast positions
    (bin units; >= 1: every position exact; 0: per-row path) and the largest
    distance between fast and exact positions found at init."""
    v, e = ctypes.c_double(), ctypes.c_double()
    _check(load().dr_geometry_position_margin(geom, ctypes.byref(v), ctypes.byref(e)))
    return v.value, e.value


def dr_geometry_free(geom: int) -> None:
    _check(load().dr_geometry_free(geom))


def dr_set_tile(geom: int, tile: Optional[Sequence[int]]) -> None:
    if tile is None:
        _check(load().dr_set_tile(geom, None))
        return
    t = dr_tile_config(*(list(tile) + [0] * (4 - len(tile))))
    _check(load().dr_set_tile(geom, ctypes.byref(t)))


def dr_autotune(geom: int, images_dev, out_dev):
    t = dr_tile_config()
    _check(load().dr_autotune(geom, ptr(images_dev), ptr(out_dev), ctypes.byref(t)))
    return t.as_tuple()


# ----------------------------------------------------------- reconstruction


def dr_reconstruct(geom: int, images, images_on_device: bool, out, totals=None, stream=None):
    _check(load().dr_reconstruct(geom, ptr(images), 1 if images_on_device else 0, ptr(out),
                                 ptr(totals), stream_handle(stream)))


def dr_reconstruct_f64(geom: int, images_dev, out, totals=None, stream=None):
    _check(load().dr_reconstruct_f64(geom, ptr(images_dev), ptr(out), ptr(totals),
                                     stream_handle(stream)))


def dr_reconstruct_noalloc(geom: int, images_dev, out, totals=None, stream=None):
    _check(load().dr_reconstruct_noalloc(geom, ptr(images_dev), ptr(out), ptr(totals),
                                         stream_handle(stream)))


def dr_debug_plan(geom: int, pixels, n_steps: int, want_bins: bool = True, want_u: bool = True,
                  edge: int = DR_EDGE_LEADING):
    pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64))
    bins = np.empty((pix.shape[0], n_steps), dtype=np.int32) if want_bins else None
    u = np.empty((pix.shape[0], n_steps), dtype=np.float64) if want_u else None
    _check(load().dr_debug_plan(geom, pix.ctypes.data, int(pix.shape[0]), int(edge), ptr(bins),
                                ptr(u)))
    return bins, u


def dr_enable_timing(geom: int, enable: bool = True) -> None:
    _check(load().dr_enable_timing(geom, 1 if enable else 0))


def dr_last_timing(geom: int):
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(load().dr_last_timing(geom, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


# ------------------------------------------------------------------ batches


def dr_batch_create(ctx: int, items, flags: int = 0) -> int:
    """items: sequence of (geom, images_dev, out_dev, totals_dev or None)."""
    arr = (dr_batch_item * len(items))()
    for i, (g, im, out, tot) in enumerate(items):
        arr[i].geom, arr[i].images, arr[i].out, arr[i].totals = g, ptr(im), ptr(out), ptr(tot)
    h = ctypes.c_void_p()
    _check(load().dr_batch_create(ctx, len(items), arr, int(flags), ctypes.byref(h)))
    return h.value


def dr_batch_run(batch: int, stream=None) -> None:
    _check(load().dr_batch_run(batch, stream_handle(stream)))


def dr_batch_tile(batch: int):
    t = dr_tile_config()
    _check(load().dr_batch_tile(batch, ctypes.byref(t)))
    return t.as_tuple()


def dr_batch_free(batch: int) -> None:
    _check(load().dr_batch_free(batch))


# ------------------------------------------------------------------ serving


def dr_submit(ctx: int, geom: int, images, images_on_device: bool, out, totals=None) -> int:
    t = ctypes.c_uint64()
    _check(load().dr_submit(ctx, geom, ptr(images), 1 if images_on_device else 0, ptr(out),
                            ptr(totals), ctypes.byref(t)))
    return t.value


def dr_poll(ctx: int, ticket: int) -> int:
    """DR_PENDING or DR_OK; raises on failure."""
    return _check(load().dr_poll(ctx, ticket), allow=(DR_OK, DR_PENDING))


def dr_wait(ctx: int, ticket: int) -> None:
    _check(load().dr_wait(ctx, ticket))


def dr_ctx_stats(ctx: int) -> dict:
    s = dr_stats()
    _check(load().dr_ctx_stats(ctx, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in dr_stats._fields_}


# ------------------------------------------------------------- pixel lists


def dr_pixel_activity(geom: int, images_dev, activity_dev, stream=None) -> None:
    _check(load().dr_pixel_activity(geom, ptr(images_dev), ptr(activity_dev),
                                    stream_handle(stream)))


def dr_select_top(geom: int, activity_dev, k: int) -> int:
    h = ctypes.c_void_p()
    _check(load().dr_select_top(geom, ptr(activity_dev), int(k), ctypes.byref(h)))
    return h.value


def dr_list_create(geom: int, pixels, on_device: bool = False) -> int:
    """pixels: int64 array (host numpy or device tensor), strictly increasing."""
    if isinstance(pixels, np.ndarray):
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pixels.shape[0]
    else:
        n = int(pixels.numel())
    h = ctypes.c_void_p()
    _check(load().dr_list_create(geom, ptr(pixels) if n else None, n, 1 if on_device else 0,
                                 ctypes.byref(h)))
    return h.value


def dr_list_size(lst: int) -> int:
    n = ctypes.c_int64()
    _check(load().dr_list_size(lst, ctypes.byref(n)))
    return n.value


def dr_list_pixels(lst: int) -> np.ndarray:
    out = np.empty(max(dr_list_size(lst), 1), dtype=np.int64)
    _check(load().dr_list_pixels(lst, ptr(out)))
    return out[:dr_list_size(lst)]


def dr_list_free(lst: int) -> None:
    _check(load().dr_list_free(lst))


def dr_reconstruct_list(lst: int, images, layout: int, images_on_device: bool, out, totals=None,
                        stream=None) -> None:
    _check(load().dr_reconstruct_list(lst, ptr(images), int(layout), 1 if images_on_device else 0,
                                      ptr(out), ptr(totals), stream_handle(stream)))


def dr_reconstruct_list_f64(lst: int, images_dev, layout: int, out, totals=None,
                            stream=None) -> None:
    _check(load().dr_reconstruct_list_f64(lst, ptr(images_dev), int(layout), ptr(out),
                                          ptr(totals), stream_handle(stream)))
