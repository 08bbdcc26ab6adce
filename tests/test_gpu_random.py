"""Seeded random scans on the GPU: each case draws the detector size, its tilt
(or an explicit, jittered pixel table), the wire axis, the number and size of
the wire steps, the depth grid (size, bin width and offset, so sweeps may lie
inside the grid or leave it at either end), the wire edge and, for some cases,
per-step monitor weights.  Every case is held to the same bar as the fixed
cases:

* the FP64-accumulation instance: bit-exact against the oracle;
* the FP32 path: |gpu - oracle| <= 1e-5 * sum_k |w_k I_k - w_{k+1} I_{k+1}| per
  pixel and bin, totals within 1e-5 of the summed scale;
* a random pixel list (full frames and a compact stack): bitwise equal to the
  dense FP32 output at those pixels.
Needs an MI355X.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_images, run_f32, run_f64

pytestmark = pytest.mark.gpu

SEEDS = list(range(24))


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


def make_case(seed):
    rng = np.random.default_rng(np.random.SeedSequence(9000 + seed))
    nx, ny = int(rng.integers(1, 140)), int(rng.integers(1, 5))
    N, B = int(rng.integers(2, 48)), int(rng.integers(1, 160))
    step = float(rng.choice([0.25, 0.5, 1.0, 2.0]))
    width = float(rng.choice([0.05, 0.3, 0.5, 1.0, 3.0]))
    s = synth.tiny(nx, ny, N, B, seed=9100 + seed, step=step, width=width,
                   n_src=int(rng.integers(1, 8)), dark=100.0, render_now=False)
    # the grid's centre: near the edge's sweep (the trailing edge runs one
    # shadow width, about 52 um, below the leading one), from below it to above
    edge = int(rng.choice([synth.EDGE_LEADING, synth.EDGE_TRAILING, synth.EDGE_BOTH]))
    mid = {synth.EDGE_LEADING: 0.0, synth.EDGE_TRAILING: -52.0, synth.EDGE_BOTH: -26.0}[edge]
    sweep = 0.5 * (N - 1) * step
    shift = mid + 0.8 * float(rng.uniform(-1.0, 1.0)) * (sweep + 0.5 * B * width)
    s.grid = synth.DepthGrid(B, s.grid.first_center + shift, width)
    kind = int(rng.integers(0, 4))
    d = s.detector
    if kind == 1:    # detector columns tilted out of x
        u = np.array([200.0, float(rng.uniform(-20, 20)), float(rng.uniform(-40, 40))])
        s.detector = synth.Detector(d.nx, d.ny, d.origin, u, d.v)
    elif kind == 2:  # wire axis tilted towards the beam and towards y
        t, p = math.radians(float(rng.uniform(-15, 15))), math.radians(float(rng.uniform(-10, 10)))
        s.wire.axis = np.array([math.cos(t) * math.cos(p), math.sin(p), math.sin(t)])
    elif kind == 3:  # explicit pixel centres, each moved a little
        x, y, z = d.pixel_xyz_arrays()
        xyz = np.stack([x, y, z], -1) + rng.uniform(-30.0, 30.0, (d.ny, d.nx, 3))
        s.detector = synth.Detector(d.nx, d.ny, d.origin, d.u, d.v, pixel_xyz=xyz)
    weights = rng.uniform(0.5, 2.0, N) if rng.uniform() < 0.3 else None
    s.wire = synth.Wire(s.wire.radius, s.wire.centers, axis=s.wire.axis, edge=edge,
                        weights=weights)
    s.name = f"random{seed}"
    synth.render(s)
    return s


def scale_of(s):
    I = s.images.astype(np.float64)
    if s.wire.weights is not None:
        I = I * s.wire.weights[:, None, None]
    return np.abs(np.diff(I, axis=0)).sum(0)


@pytest.mark.parametrize("seed", SEEDS)
def test_random_scan(dr, ctx, seed):
    import torch
    s = make_case(seed)
    ref, tref, _ = oracle.reconstruct(s)
    out64, _ = run_f64(dr, ctx, s)
    assert np.array_equal(out64.view(np.int64), ref.view(np.int64)), seed
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        out, tot = run_f32(dr, ctx, s, geom=g)
        scale = scale_of(s)
        assert not np.isnan(out).any()
        assert np.all(np.abs(out.astype(np.float64) - ref) <= 1e-5 * scale[None]), seed
        assert np.all(np.abs(tot.astype(np.float64) - tref) <= 1e-5 * max(scale.sum(), 1.0))
        # a random list of pixels, as full frames and as a compact stack
        npix = s.detector.nx * s.detector.ny
        rng = np.random.default_rng(seed)
        pix = np.unique(rng.integers(0, npix, max(1, npix // 3)))
        lst = dr.dr_list_create(g, pix)
        try:
            B, N, n = s.grid.n_bins, s.wire.n_steps, pix.shape[0]
            flat = out.reshape(B, -1)
            compact = np.ascontiguousarray(s.images.reshape(N, -1)[:, pix])
            for layout, img in ((dr.DR_LAYOUT_FULL, s.images), (dr.DR_LAYOUT_LIST, compact)):
                o = torch.full((B, n), float("nan"), device="cuda")
                dr.dr_reconstruct_list(lst, dev_images(img), layout, True, o, None,
                                       torch.cuda.current_stream())
                torch.cuda.synchronize()
                assert np.array_equal(o.cpu().numpy(), flat[:, pix]), (seed, layout)
        finally:
            dr.dr_list_free(lst)
    finally:
        dr.dr_geometry_free(g)
