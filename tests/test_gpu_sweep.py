"""Device square root and division, swept through the tangent depth (needs an
MI355X).

Every wire position u_k = (d_k - e0) / width rests on one correctly rounded
square root and one correctly rounded division per (pixel, step) (the
cancellation-free tangent form); any difference between the device's and the
host's results shows up in the bits of u_k.  This test draws randomised
geometries (flat detector, tilted detector, tilted wire axis, an explicit
jittered pixel table; detector distance, wire height, radius, scan direction
and step size across the ranges of the oracle's pins), asks the library for
u_k of random pixels over 1001 steps on both wire edges, and requires every
value to equal the oracle's bit for bit: at least 10^8 evaluations in total.
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

N_STEPS = 1001
PIXELS_PER_CASE = 9000
KINDS = ("flat", "tilted_detector", "tilted_axis", "pixel_table", "flat", "tilted_axis")
_count = {"evaluations": 0}


@pytest.fixture(scope="module")
def dr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2201_13309_amd import dr as d
    d.load()
    return d


@pytest.fixture(scope="module")
def ctx(dr):
    h = dr.dr_ctx_create(0, 0)
    yield h
    dr.dr_ctx_destroy(h)


def make_geometry(case):
    rng = np.random.default_rng(np.random.SeedSequence(4400 + case))
    kind = KINDS[case]
    distance_mm = float(rng.uniform(150.0, 800.0))
    pitch = float(rng.choice([50.0, 100.0, 200.0, 400.0]))
    side = 256 if kind == "pixel_table" else 2048
    det = synth.flat_detector(side, side, pitch, distance_mm)
    if kind == "tilted_detector":
        u = np.array([pitch, rng.uniform(-0.2, 0.2) * pitch, rng.uniform(-0.2, 0.2) * pitch])
        det = synth.Detector(det.nx, det.ny, det.origin, u, det.v)
    elif kind == "pixel_table":
        x, y, z = det.pixel_xyz_arrays()
        xyz = np.stack([x, y, z], -1) + rng.uniform(-0.4 * pitch, 0.4 * pitch, (side, side, 3))
        det = synth.Detector(det.nx, det.ny, det.origin, det.u, det.v, pixel_xyz=xyz)
    step = float(rng.uniform(0.1, 1.0))
    theta = math.radians(float(rng.uniform(20.0, 70.0)))
    radius = float(rng.uniform(5.0, 100.0))
    mid_y = float(rng.uniform(600.0, 2000.0))
    mid_z = float(rng.uniform(-300.0, 300.0))
    k = np.arange(N_STEPS, dtype=np.float64) - (N_STEPS - 1) / 2.0
    centers = np.zeros((N_STEPS, 3))
    centers[:, 1] = mid_y + k * step * math.cos(theta)
    centers[:, 2] = mid_z + k * step * math.sin(theta)
    axis = np.array([1.0, 0.0, 0.0])
    if kind == "tilted_axis":
        t = math.radians(float(rng.uniform(-15.0, 15.0)))
        p = math.radians(float(rng.uniform(-10.0, 10.0)))
        axis = np.array([math.cos(t) * math.cos(p), math.sin(p), math.sin(t)])
    width = float(rng.choice([0.1, 0.5, 1.0]))
    grid = synth.centered_grid(int(rng.integers(101, 1002)), width)
    npix = det.nx * det.ny
    pix = np.unique(np.concatenate([[0, det.nx - 1, npix - det.nx, npix - 1],
                                    rng.integers(0, npix, PIXELS_PER_CASE)]))
    return kind, det, radius, centers, axis, grid, pix


@pytest.mark.parametrize("case", range(len(KINDS)))
def test_tangent_positions_bitwise(dr, ctx, case):
    kind, det, radius, centers, axis, grid, pix = make_geometry(case)
    wire_both = synth.Wire(radius, centers, axis=axis, edge=synth.EDGE_BOTH)
    g = dr.dr_geometry_init(ctx, det, wire_both, grid)
    try:
        for edge in (synth.EDGE_LEADING, synth.EDGE_TRAILING):
            scan = synth.Scan(f"sweep{case}", det, synth.Wire(radius, centers, axis=axis, edge=edge),
                              grid, None, 0.0, False, 0)
            _, bins_ref, u_ref = oracle.reconstruct_pixels(scan, pix, want_bins=True, want_u=True)
            bins, u = dr.dr_debug_plan(g, pix, N_STEPS, edge=edge)
            assert np.all(np.isfinite(u_ref))
            diff = u.view(np.int64) != u_ref.view(np.int64)
            assert not diff.any(), (
                f"{kind} case {case} edge {edge}: {int(diff.sum())} of {diff.size} positions "
                f"differ, e.g. pixel {pix[np.nonzero(diff)[0][0]]}")
            assert np.array_equal(bins, bins_ref)
            _count["evaluations"] += u.size
    finally:
        dr.dr_geometry_free(g)


def test_sweep_count():
    """The sweep holds at least 10^8 tangent evaluations (one square root and
    one division each); after the cases above have run, all of them were
    compared."""
    planned = sum(2 * N_STEPS * make_geometry(c)[-1].shape[0] for c in range(len(KINDS)))
    n = _count["evaluations"]
    print(f"tangent evaluations compared bit for bit: {n:,} of {planned:,}")
    assert planned >= 10 ** 8, planned
    assert n in (0, planned), (n, planned)
