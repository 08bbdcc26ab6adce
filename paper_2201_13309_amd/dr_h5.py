"""ctypes binding of the HDF5 file layer (include/dr_h5.h, libdr_h5.so).

Argument marshalling only.  The library exists where an HDF5 installation was
found at build time; load() raises ImportError otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from .dr import DRError, DR_OK, ptr

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdr_h5.so")

ABI_SYMBOLS = (
    "dr_h5_open_stack", "dr_h5_stack_shape", "dr_h5_read_rows", "dr_h5_close_stack",
    "dr_h5_read_scalars", "dr_h5_write_stack", "dr_h5_write_scalars",
    "dr_h5_write_depth_images", "dr_h5_last_error",
)

_lib = None


def load(path: Optional[str] = None):
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libdr_h5.so not built ({p}); it needs an HDF5 installation")
    lib = ctypes.CDLL(p)
    vp, i32, pp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p)
    P = ctypes.POINTER
    sigs = {
        "dr_h5_open_stack": [pp, i32, ctypes.c_char_p, P(vp)],
        "dr_h5_stack_shape": [vp, P(i32), P(i32), P(i32), P(i32)],
        "dr_h5_read_rows": [vp, i32, i32, vp, i32],
        "dr_h5_close_stack": [vp],
        "dr_h5_read_scalars": [pp, i32, ctypes.c_char_p, vp],
        "dr_h5_write_stack": [pp, i32, ctypes.c_char_p, vp, i32, i32, i32],
        "dr_h5_write_scalars": [pp, i32, ctypes.c_char_p, vp],
        "dr_h5_write_depth_images": [ctypes.c_char_p, ctypes.c_char_p, vp, i32, i32, i32,
                                     ctypes.c_double, ctypes.c_double],
    }
    for name, argt in sigs.items():
        f = getattr(lib, name)
        f.argtypes = argt
        f.restype = ctypes.c_int32
    lib.dr_h5_last_error.argtypes = []
    lib.dr_h5_last_error.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != DR_OK:
        raise DRError(rc, load().dr_h5_last_error().decode(errors="replace"))


def _paths(paths: Sequence[str]):
    arr = (ctypes.c_char_p * len(paths))(*[os.fsencode(p) for p in paths])
    return arr


def open_stack(paths: Sequence[str], dataset: str) -> int:
    h = ctypes.c_void_p()
    _check(load().dr_h5_open_stack(_paths(paths), len(paths), dataset.encode(), ctypes.byref(h)))
    return h.value


def stack_shape(stack: int):
    """(n_files, ny, nx, direct_files)."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(load().dr_h5_stack_shape(stack, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def read_rows(stack: int, row0: int, nrows: int, out, nthreads: int = 0) -> None:
    """out: uint16/int16 host buffer [n_files][nrows][nx] (numpy or pinned tensor)."""
    _check(load().dr_h5_read_rows(stack, int(row0), int(nrows), ptr(out), int(nthreads)))


def close_stack(stack: int) -> None:
    _check(load().dr_h5_close_stack(stack))


def read_scalars(paths: Sequence[str], dataset: str) -> np.ndarray:
    out = np.empty(len(paths), dtype=np.float64)
    _check(load().dr_h5_read_scalars(_paths(paths), len(paths), dataset.encode(), ptr(out)))
    return out


def write_stack(paths: Sequence[str], dataset: str, images: np.ndarray, deflate: int = 0) -> None:
    im = np.ascontiguousarray(images).view(np.uint16)
    assert im.ndim == 3 and im.shape[0] == len(paths)
    _check(load().dr_h5_write_stack(_paths(paths), len(paths), dataset.encode(), ptr(im),
                                    im.shape[1], im.shape[2], int(deflate)))


def write_scalars(paths: Sequence[str], dataset: str, values) -> None:
    v = np.ascontiguousarray(values, dtype=np.float64)
    _check(load().dr_h5_write_scalars(_paths(paths), len(paths), dataset.encode(), ptr(v)))


def write_depth_images(path: str, dataset: str, images, first_center: float,
                       width: float) -> None:
    """images: float32 [n_bins][ny][nx] on the host (numpy or CPU tensor)."""
    if isinstance(images, np.ndarray):
        images = np.ascontiguousarray(images, dtype=np.float32)
        shape = images.shape
    else:
        shape = tuple(images.shape)
    _check(load().dr_h5_write_depth_images(os.fsencode(path), dataset.encode(), ptr(images),
                                           shape[0], shape[1], shape[2], float(first_center),
                                           float(width)))
