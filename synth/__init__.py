"""Seeded synthetic workloads for wire-scan depth reconstruction.

Input generation only: this package is shared by the tests, the benchmark and
the smoke check, and it holds none of the reconstruction arithmetic (no
tangent depths, bin indices or overlap fractions).  It builds

* the instrument geometry of each workload (detector pixel grid, wire
  positions, depth grid), with every coordinate built from exact products so
  that pixels of one detector row share bit-identical (y, z) centres;
* the forward model: point sources on the beam, rays to detector spots,
  occlusion by the wire disc, Poisson counts (``forward.c``).

The workloads follow the paper's problem statement (an image stack of p images
of m x n pixels, Sec. III-B) at the sizes of the benchmark configurations.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

UM_PER_MM = 1000.0


def build(force: bool = True) -> str:
    """Compile forward.c into libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               os.path.join(_HERE, "forward.c"), "-o", LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        d, i32, i64, u64, p = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                               ctypes.c_uint64, ctypes.c_void_p)
        lib.synth_render.argtypes = [i32, i32, p, p, p, i32, p, p, p, p, d, p, p, p, d, i32, u64,
                                     p, i32]
        lib.synth_render.restype = ctypes.c_int
        lib.synth_uniforms.argtypes = [u64, u64, u64, i64, p]
        lib.synth_uniforms.restype = None
        lib.synth_occluded.argtypes = [d, d, d, d, d, d]
        lib.synth_occluded.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# ---------------------------------------------------------------- geometry


@dataclass
class Detector:
    """Pixel (j, i) centre = (origin + i*u) + j*v in um; i = column, j = row."""
    nx: int
    ny: int
    origin: np.ndarray
    u: np.ndarray
    v: np.ndarray
    pixel_xyz: Optional[np.ndarray] = None  # optional [ny][nx][3] override

    def pixel_xyz_arrays(self):
        """Pixel-centre (x, y, z) arrays [ny][nx] for the forward model."""
        if self.pixel_xyz is not None:
            return tuple(np.ascontiguousarray(self.pixel_xyz[..., q]) for q in range(3))
        i = np.arange(self.nx, dtype=np.float64)[None, :]
        j = np.arange(self.ny, dtype=np.float64)[:, None]
        return tuple(np.ascontiguousarray(np.broadcast_to(
            (self.origin[q] + i * self.u[q]) + j * self.v[q], (self.ny, self.nx)))
            for q in range(3))

    def pixel_yz(self):
        """Pixel-centre (y, z) arrays [ny][nx]."""
        _, y, z = self.pixel_xyz_arrays()
        return y, z


EDGE_LEADING, EDGE_TRAILING, EDGE_BOTH = 0, 1, 2


@dataclass
class Wire:
    radius: float
    centers: np.ndarray  # [n_steps][3] um
    axis: np.ndarray = field(default_factory=lambda: np.array([1.0, 0.0, 0.0]))
    edge: int = EDGE_LEADING  # which wire edge the reconstruction uses
    weights: Optional[np.ndarray] = None  # per-step sample weights (monitor normalisation)

    @property
    def n_steps(self) -> int:
        return int(self.centers.shape[0])


@dataclass
class DepthGrid:
    """Bin b is centred at first_center + b*width (um)."""
    n_bins: int
    first_center: float
    width: float


@dataclass
class Sources:
    zs: np.ndarray      # depth on the beam, um
    ci: np.ndarray      # spot centre column (pixel units, continuous)
    cj: np.ndarray      # spot centre row
    amp: np.ndarray     # peak expected counts
    sigma: float = 1.5  # Gaussian spot width in pixels; 0 = single pixel
    trunc: float = 4.0  # spot truncation radius in pixels


@dataclass
class Scan:
    name: str
    detector: Detector
    wire: Wire
    grid: DepthGrid
    sources: Sources
    dark: float
    noise: bool
    seed: int
    images: Optional[np.ndarray] = None  # uint16 [n_steps][ny][nx]

    @property
    def pixel_steps(self) -> int:
        return self.detector.nx * self.detector.ny * self.wire.n_steps


def flat_detector(nx: int, ny: int, pitch: float, distance_mm: float = 510.0,
                  full_nx: Optional[int] = None, full_ny: Optional[int] = None,
                  i0: int = 0, j0: int = 0) -> Detector:
    """Detector normal to y at `distance_mm`, 90 deg take-off, centred on the
    beam.  Columns run along +x and rows along +z.  An ROI is the (i0, j0)
    sub-window of a full_nx x full_ny detector of the same pitch.  All
    coordinates are exact multiples of half a pitch, built without trig."""
    fnx = nx if full_nx is None else full_nx
    fny = ny if full_ny is None else full_ny
    ox = -(fnx - 1) / 2.0 * pitch + i0 * pitch
    oz = -(fny - 1) / 2.0 * pitch + j0 * pitch
    origin = np.array([ox, distance_mm * UM_PER_MM, oz], dtype=np.float64)
    u = np.array([pitch, 0.0, 0.0], dtype=np.float64)
    v = np.array([0.0, 0.0, pitch], dtype=np.float64)
    return Detector(nx, ny, origin, u, v)


def wire_scan(n_steps: int, step: float, radius: float = 26.0,
              mid_yz=(300.0, -26.0)) -> Wire:
    """Wire centres C_k = mid + (k - (N-1)/2) * step * (0, sqrt(1/2), sqrt(1/2)):
    a 45 deg scan, up and downstream, centred so that the leading edge seen
    from the detector centre sits near depth 0 at mid-scan."""
    h = math.sqrt(0.5)
    k = np.arange(n_steps, dtype=np.float64) - (n_steps - 1) / 2.0
    c = np.zeros((n_steps, 3), dtype=np.float64)
    c[:, 1] = mid_yz[0] + k * step * h
    c[:, 2] = mid_yz[1] + k * step * h
    return Wire(radius=radius, centers=c)


def centered_grid(n_bins: int, width: float) -> DepthGrid:
    return DepthGrid(n_bins=n_bins, first_center=-(n_bins - 1) / 2.0 * width, width=width)


# ------------------------------------------------------------- forward model


def draw_sources(rng: np.random.Generator, n: int, nx: int, ny: int, zlo: float, zhi: float,
                 amp_lo: float = 2e3, amp_hi: float = 2e4, sigma: float = 1.5,
                 trunc: float = 4.0, integer_amp: bool = False) -> Sources:
    zs = rng.uniform(zlo, zhi, n)
    ci = rng.uniform(0.0, nx - 1.0, n)
    cj = rng.uniform(0.0, ny - 1.0, n)
    amp = rng.uniform(amp_lo, amp_hi, n)
    if integer_amp:
        amp = np.floor(amp)
    return Sources(zs=zs, ci=ci, cj=cj, amp=amp, sigma=sigma, trunc=trunc)


def contributions(src: Sources, nx: int, ny: int):
    """CSR over pixels of (expected counts, source depth) pairs."""
    pix: List[np.ndarray] = []
    gain: List[np.ndarray] = []
    zsl: List[np.ndarray] = []
    if src.sigma <= 0.0:
        ii = np.clip(np.rint(src.ci).astype(np.int64), 0, nx - 1)
        jj = np.clip(np.rint(src.cj).astype(np.int64), 0, ny - 1)
        pix.append(jj * nx + ii)
        gain.append(src.amp.astype(np.float64))
        zsl.append(src.zs.astype(np.float64))
    else:
        R = int(math.ceil(src.trunc)) + 1
        off = np.arange(-R, R + 1)
        for dj in off:
            for di in off:
                ii = np.floor(src.ci).astype(np.int64) + di
                jj = np.floor(src.cj).astype(np.int64) + dj
                d2 = (ii - src.ci) ** 2 + (jj - src.cj) ** 2
                ok = (d2 <= src.trunc ** 2) & (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
                if not ok.any():
                    continue
                pix.append((jj * nx + ii)[ok])
                gain.append((src.amp * np.exp(-d2 / (2.0 * src.sigma ** 2)))[ok])
                zsl.append(src.zs[ok])
    pix_a = np.concatenate(pix) if pix else np.zeros(0, np.int64)
    gain_a = np.concatenate(gain) if gain else np.zeros(0)
    zs_a = np.concatenate(zsl) if zsl else np.zeros(0)
    order = np.argsort(pix_a, kind="stable")
    pix_a, gain_a, zs_a = pix_a[order], gain_a[order], zs_a[order]
    counts = np.bincount(pix_a, minlength=nx * ny)
    ptr = np.zeros(nx * ny + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, np.ascontiguousarray(gain_a), np.ascontiguousarray(zs_a)


def render(scan: Scan, out: Optional[np.ndarray] = None, nthreads: int = 0) -> np.ndarray:
    """Fill scan.images (uint16 [N][ny][nx]) with the forward model."""
    det, wire = scan.detector, scan.wire
    px, py, pz = det.pixel_xyz_arrays()
    ptr, gain, zs = contributions(scan.sources, det.nx, det.ny)
    N = wire.n_steps
    if out is None:
        out = np.empty((N, det.ny, det.nx), dtype=np.uint16)
    assert out.dtype == np.uint16 and out.shape == (N, det.ny, det.nx) and out.flags.c_contiguous
    cx = np.ascontiguousarray(wire.centers[:, 0])
    cy = np.ascontiguousarray(wire.centers[:, 1])
    cz = np.ascontiguousarray(wire.centers[:, 2])
    axis = np.asarray(wire.axis, dtype=np.float64)
    axis = np.ascontiguousarray(axis / np.linalg.norm(axis))
    if nthreads <= 0:
        nthreads = min(16, os.cpu_count() or 1)
    _load().synth_render(det.nx, det.ny, _ptr(px), _ptr(py), _ptr(pz), N, _ptr(cx), _ptr(cy),
                         _ptr(cz), _ptr(axis), float(wire.radius), _ptr(ptr), _ptr(gain), _ptr(zs),
                         float(scan.dark), 1 if scan.noise else 0,
                         int(scan.seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out), int(nthreads))
    scan.images = out
    return out


def occluded(zs: float, py: float, pz: float, cy: float, cz: float, r: float) -> bool:
    """The forward model's occlusion predicate (strict: distance < r)."""
    return bool(_load().synth_occluded(zs, py, pz, cy, cz, r))


def philox_uniforms(seed: int, a: int, b: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_uniforms(seed, a, b, n, _ptr(out))
    return out


# --------------------------------------------------------------- workloads


def config1(seed: int = 1, noise: bool = True, render_now: bool = True) -> Scan:
    """64x64 px at 200 um, 510 mm, 90 deg; wire r = 26 um stepped 41 x 1 um at
    45 deg; 101 bins of 1 um over [-50, 50]; 8 sources, dark 0."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    det = flat_detector(64, 64, 200.0)
    wire = wire_scan(41, 1.0)
    grid = centered_grid(101, 1.0)
    src = draw_sources(rng, 8, 64, 64, -13.0, 13.0)
    s = Scan("config1", det, wire, grid, src, dark=0.0, noise=noise, seed=seed)
    if render_now:
        render(s)
    return s


def config2(seed: int = 2, render_now: bool = True, nthreads: int = 0) -> Scan:
    """1024x1024 px (2x2-binned geometry, 400 um), 401 steps x 0.5 um, 501 bins
    x 0.5 um, 2000 sources at depths U(-120, 120), dark 100, Poisson."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    det = flat_detector(1024, 1024, 400.0)
    wire = wire_scan(401, 0.5)
    grid = centered_grid(501, 0.5)
    src = draw_sources(rng, 2000, 1024, 1024, -120.0, 120.0)
    s = Scan("config2", det, wire, grid, src, dark=100.0, noise=True, seed=seed)
    if render_now:
        render(s, nthreads=nthreads)
    return s


def config3(seed: int = 3, render_now: bool = True, out: Optional[np.ndarray] = None,
            nthreads: int = 0) -> Scan:
    """2048x2048 px at 200 um, 1001 steps x 0.5 um, 1001 bins x 0.5 um, 20000
    sources at depths U(-170, 170), dark 100, Poisson (8.4 GB of uint16)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    det = flat_detector(2048, 2048, 200.0)
    wire = wire_scan(1001, 0.5)
    grid = centered_grid(1001, 0.5)
    src = draw_sources(rng, 20000, 2048, 2048, -170.0, 170.0)
    s = Scan("config3", det, wire, grid, src, dark=100.0, noise=True, seed=seed)
    if render_now:
        render(s, out=out, nthreads=nthreads)
    return s


def config4(seed: int = 4, render_now: bool = True, n_scans: int = 16,
            nthreads: int = 0) -> List[Scan]:
    """16 scans of uneven size: ROI side in {256, 512, 768, 1024} (sub-window of
    the 2048^2 / 200 um detector at a seeded offset), steps U{101..801} x 0.5 um,
    bins U{201..801} x 0.5 um centred on 0, 2000*(side/1024)^2 sources, dark 100."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss)
    scans = []
    for n in range(n_scans):
        side = int(rng.choice([256, 512, 768, 1024]))
        N = int(rng.integers(101, 802))
        B = int(rng.integers(201, 802))
        i0 = int(rng.integers(0, 2048 - side + 1))
        j0 = int(rng.integers(0, 2048 - side + 1))
        det = flat_detector(side, side, 200.0, full_nx=2048, full_ny=2048, i0=i0, j0=j0)
        wire = wire_scan(N, 0.5)
        grid = centered_grid(B, 0.5)
        half = 0.5 * min((N - 1) * 0.5 * 0.7, (B - 2) * 0.5)
        nsrc = max(1, int(round(2000 * (side / 1024.0) ** 2)))
        src = draw_sources(rng, nsrc, side, side, -half, half)
        s = Scan(f"config4[{n}]", det, wire, grid, src, dark=100.0, noise=True,
                 seed=int(seed * 1000 + n))
        if render_now:
            render(s, nthreads=nthreads)
        scans.append(s)
    return scans


def tiny(nx: int, ny: int, n_steps: int, n_bins: int, seed: int = 7, pitch: float = 200.0,
         step: float = 1.0, width: float = 1.0, n_src: int = 4, dark: float = 0.0,
         noise: bool = True, sigma: float = 1.5, zlo: Optional[float] = None,
         zhi: Optional[float] = None, integer_amp: bool = False,
         render_now: bool = True) -> Scan:
    """Small seeded scan for parity and edge-case tests (ragged sizes allowed)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    det = flat_detector(nx, ny, pitch)
    wire = wire_scan(n_steps, step)
    grid = centered_grid(n_bins, width)
    sweep = 0.5 * (n_steps - 1) * step * 0.7
    lo = -sweep if zlo is None else zlo
    hi = sweep if zhi is None else zhi
    src = draw_sources(rng, n_src, nx, ny, lo, hi, sigma=sigma, integer_amp=integer_amp)
    s = Scan(f"tiny{nx}x{ny}x{n_steps}", det, wire, grid, src, dark=dark, noise=noise, seed=seed)
    if render_now:
        render(s)
    return s


def poisson_arrivals(seed: int, rate_hz: float, n: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process: exponential gaps at `rate_hz`."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))
