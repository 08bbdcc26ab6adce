"""ORACLE - test infrastructure only.

ctypes binding of ``oracle.c``: the plain FP64 CPU reconstruction used by the
tests, the smoke check and the benchmark's CPU baseline.  Nothing in the
product imports this package; it imports nothing from the product.

Scan arguments are duck-typed: any object with ``detector`` (nx, ny, origin,
u, v, pixel_xyz), ``wire`` (radius, centers) and ``grid`` (n_bins,
first_center, width) attributes works.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]

_libs = {}


def build(force: bool = True, src: Optional[str] = None, out: Optional[str] = None) -> str:
    """Compile the oracle (gcc, -O2 -ffp-contract=off, OpenMP)."""
    src = src or os.path.join(_HERE, "oracle.c")
    out = out or LIB_PATH
    if force or not os.path.exists(out):
        subprocess.check_call(["gcc", *CFLAGS, src, "-o", out + ".tmp", "-lm"])
        os.replace(out + ".tmp", out)
    return out


def load(path: Optional[str] = None):
    path = path or LIB_PATH
    if path not in _libs:
        if path == LIB_PATH and not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        d, i32, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_tangent_depth.argtypes = [d, d, d, d, d, i32]
        lib.oracle_tangent_depth.restype = d
        lib.oracle_edge_sign.argtypes = [d, d, i32, p, d]
        lib.oracle_edge_sign.restype = i32
        lib.oracle_bin_profile.argtypes = [p, p, i32, i32, i32, p, i64]
        lib.oracle_bin_profile.restype = None
        lib.oracle_reconstruct.argtypes = [i32, i32, p, p, p, p, d, p, i32, p, i32, d, d, i32,
                                           p, p, i32, i32, p, p, p, i32]
        lib.oracle_reconstruct.restype = i32
        lib.oracle_reconstruct_pixels.argtypes = [i32, i32, p, p, p, p, d, p, i32, p, i32, d, d,
                                                  i32, p, p, p, i64, p, p, p, i32]
        lib.oracle_reconstruct_pixels.restype = i32
        lib.oracle_activity.argtypes = [p, i32, i64, p]
        lib.oracle_activity.restype = None
        lib.oracle_select_top.argtypes = [p, i64, i64, p]
        lib.oracle_select_top.restype = i32
        _libs[path] = lib
    return _libs[path]


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class OracleError(RuntimeError):
    pass


def tangent_depth(py, pz, cy, cz, r, s, lib=None) -> float:
    return (lib or load()).oracle_tangent_depth(float(py), float(pz), float(cy), float(cz),
                                                float(r), int(s))


def edge_sign(py, pz, centers, r, lib=None) -> int:
    """Leading side for a pixel at (y, z) and wire centres [N][3] with the wire
    axis along x (the projection is then (eta, xi) = (y, z))."""
    c = _f64(centers)
    wyz = np.ascontiguousarray(c[:, 1:3])
    return (lib or load()).oracle_edge_sign(float(py), float(pz), wyz.shape[0], _p(wyz), float(r))


EDGE_LEADING, EDGE_TRAILING, EDGE_BOTH = 0, 1, 2


def bin_profile(u, intensities, n_bins: int, trailing: bool = False, lib=None) -> np.ndarray:
    """Binning of one pixel given its positions u_k (bin units) and counts;
    trailing=True takes dI_k = I_{k+1} - I_k."""
    u = _f64(u)
    I = _f64(intensities)
    assert u.shape == I.shape and u.ndim == 1
    out = np.zeros(n_bins, dtype=np.float64)
    (lib or load()).oracle_bin_profile(_p(u), _p(I), u.shape[0], int(n_bins), 1 if trailing else 0,
                                       _p(out), 1)
    return out


def _geom_args(scan):
    det, wire, grid = scan.detector, scan.wire, scan.grid
    origin, u, v = _f64(det.origin), _f64(det.u), _f64(det.v)
    pxyz = None if det.pixel_xyz is None else _f64(det.pixel_xyz)
    centers = _f64(wire.centers)
    axis = _f64(getattr(wire, "axis", (1.0, 0.0, 0.0)))
    w = getattr(wire, "weights", None)
    w = None if w is None else _f64(w)
    assert w is None or w.shape == (centers.shape[0],)
    keep = (origin, u, v, pxyz, centers, axis, w)
    args = (int(det.nx), int(det.ny), _p(origin), _p(u), _p(v), _p(pxyz), float(wire.radius),
            _p(axis), int(centers.shape[0]), _p(centers), int(grid.n_bins),
            float(grid.first_center), float(grid.width), int(getattr(wire, "edge", EDGE_LEADING)),
            _p(w))
    return args, keep


def reconstruct(scan, images: Optional[np.ndarray] = None, row0: int = 0,
                nrows: Optional[int] = None, want_bins: bool = False, nthreads: int = 0,
                lib=None):
    """FP64 reconstruction of rows [row0, row0+nrows).

    Returns (out [n_bins][nrows][nx] f64, totals [n_bins] f64, bins or None)."""
    images = scan.images if images is None else images
    images = np.ascontiguousarray(images, dtype=np.uint16)
    det, grid = scan.detector, scan.grid
    nrows = det.ny - row0 if nrows is None else nrows
    N = scan.wire.centers.shape[0]
    assert images.shape == (N, det.ny, det.nx)
    out = np.empty((grid.n_bins, nrows, det.nx), dtype=np.float64)
    tot = np.empty(grid.n_bins, dtype=np.float64)
    bins = np.empty((nrows * det.nx, N), dtype=np.int32) if want_bins else None
    args, keep = _geom_args(scan)
    rc = (lib or load()).oracle_reconstruct(*args, _p(images), int(row0), int(nrows), _p(out),
                                            _p(tot), _p(bins), int(nthreads))
    del keep
    if rc != 0:
        raise OracleError(f"oracle_reconstruct failed ({rc})")
    return out, tot, bins


def reconstruct_pixels(scan, pixels, images: Optional[np.ndarray] = None,
                       want_bins: bool = True, want_u: bool = False, nthreads: int = 0,
                       lib=None):
    """FP64 profiles of listed pixels (flat j*nx+i); with no images (neither
    given nor held by the scan) only the positions.

    Returns (out [npix][n_bins], bins [npix][N] or None, u [npix][N] or None)."""
    pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64))
    N = scan.wire.centers.shape[0]
    B = scan.grid.n_bins
    images = scan.images if images is None else images
    if images is not None:
        images = np.ascontiguousarray(images, dtype=np.uint16)
    out = np.empty((pix.shape[0], B), dtype=np.float64)
    bins = np.empty((pix.shape[0], N), dtype=np.int32) if want_bins else None
    upos = np.empty((pix.shape[0], N), dtype=np.float64) if want_u else None
    args, keep = _geom_args(scan)
    rc = (lib or load()).oracle_reconstruct_pixels(*args, _p(images), _p(pix),
                                                   pix.shape[0], _p(out), _p(bins), _p(upos),
                                                   int(nthreads))
    del keep
    if rc != 0:
        raise OracleError(f"oracle_reconstruct_pixels failed ({rc})")
    return out, bins, upos


def activity(images: np.ndarray, lib=None) -> np.ndarray:
    """Pixel activity sum_k |I_k - I_{k+1}| of a stack [N][ny][nx] (or
    [N][npix]), flat over pixels, uint64."""
    im = np.ascontiguousarray(images, dtype=np.uint16)
    N = im.shape[0]
    npix = int(np.prod(im.shape[1:]))
    out = np.empty(npix, dtype=np.uint64)
    (lib or load()).oracle_activity(_p(im), N, npix, _p(out))
    return out


def select_top(act: np.ndarray, k: int, lib=None) -> np.ndarray:
    """The k pixels of largest activity, ties to the lower index, in
    increasing index order (int64)."""
    a = np.ascontiguousarray(act, dtype=np.uint64)
    out = np.empty(max(int(k), 1), dtype=np.int64)
    rc = (lib or load()).oracle_select_top(_p(a), a.shape[0], int(k), _p(out))
    if rc != 0:
        raise OracleError(f"oracle_select_top failed ({rc})")
    return out[:int(k)].copy()
