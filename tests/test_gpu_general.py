"""General geometry on the GPU: a detector whose rows do not share one
projected position, explicit per-pixel centres and wire axes off the lab x
axis (the projection onto the plane normal to the axis).  Such geometries take
the per-pixel path; it is held to the same bar as the per-row path:

* bin indices floor(u_k) and positions u_k: bit-exact against the oracle;
* the FP64-accumulation instance: bit-exact output;
* the FP32 path: |gpu - oracle| <= 1e-5 * sum_k |I_k - I_{k+1}| per pixel and
  bin, totals within 1e-5 of the summed scale;
* host-image slab streaming: bitwise equal to the device-resident run.
Needs an MI355X.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_f32_close, assert_totals_close, run_f32, run_f64

pytestmark = pytest.mark.gpu


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


def _tilted_detector(s, u):
    d = s.detector
    s.detector = synth.Detector(d.nx, d.ny, d.origin, np.asarray(u, dtype=np.float64), d.v)
    return s


def _cover(s, lo=-72.0, hi=24.0):
    """Spread the scan's bins over [lo, hi] um, which holds the sweeps of both
    wire edges for these scans (sources near depth 0)."""
    w = (hi - lo) / s.grid.n_bins
    s.grid = synth.DepthGrid(s.grid.n_bins, lo + 0.5 * w, w)


def make_case(name):
    if name == "tilted_detector":  # columns leave the x axis; ragged second tile per row
        s = synth.tiny(300, 4, 31, 81, seed=201, n_src=10, dark=100.0, render_now=False)
        _tilted_detector(s, [200.0, 15.0, 35.0])
    elif name == "axis_xz":        # wire axis tilted 12 degrees towards the beam
        s = synth.tiny(80, 5, 33, 91, seed=202, n_src=8, dark=100.0, render_now=False)
        t = math.radians(12.0)
        s.wire.axis = np.array([math.cos(t), 0.0, math.sin(t)])
    elif name == "axis_xy":        # tilted 7 degrees towards y, given unnormalised
        s = synth.tiny(72, 6, 29, 71, seed=203, n_src=8, dark=100.0, render_now=False)
        t = math.radians(7.0)
        s.wire.axis = np.array([3.0 * math.cos(t), 3.0 * math.sin(t), 0.0])
    elif name == "axis_oblique":   # tilted in x, y and z, with a tilted detector
        s = synth.tiny(64, 7, 27, 81, seed=204, n_src=8, dark=100.0, render_now=False)
        a = np.array([1.0, 0.12, -0.2])
        s.wire.axis = a / np.linalg.norm(a)
        _tilted_detector(s, [200.0, -10.0, 20.0])
    elif name == "pixel_table_jitter":  # explicit centres, each moved a little
        s = synth.tiny(48, 5, 21, 61, seed=205, n_src=6, dark=100.0, render_now=False)
        x, y, z = s.detector.pixel_xyz_arrays()
        rng = np.random.default_rng(205)
        xyz = np.stack([x, y, z], -1) + rng.uniform(-20.0, 20.0, (5, 48, 3))
        d = s.detector
        s.detector = synth.Detector(d.nx, d.ny, d.origin, d.u, d.v, pixel_xyz=xyz)
    elif name == "tilted_non_monotone":  # forward, then part of the way back: bins revisited
        s = synth.tiny(96, 4, 25, 81, seed=206, n_src=8, dark=100.0, render_now=False)
        _tilted_detector(s, [200.0, 5.0, 30.0])
        c = s.wire.centers
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(
            np.concatenate([c, c[::-1][1:10]], axis=0)))
    elif name == "tilted_coarse":  # intervals spanning many bins
        s = synth.tiny(64, 3, 12, 300, seed=207, n_src=6, dark=100.0, step=4.0, width=0.1,
                       render_now=False)
        _tilted_detector(s, [200.0, 0.0, 25.0])
    elif name == "tilted_decreasing":  # scanned backwards
        s = synth.tiny(128, 3, 41, 101, seed=208, n_src=8, dark=100.0, render_now=False)
        _tilted_detector(s, [200.0, 0.0, -30.0])
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(s.wire.centers[::-1]))
    elif name == "tilted_many_bins":  # partial totals too large for LDS: summed in place
        s = synth.tiny(40, 2, 21, 20000, seed=209, n_src=4, dark=100.0, width=0.002,
                       render_now=False)
        _tilted_detector(s, [200.0, 0.0, 10.0])
    elif name == "tilted_repeated_steps":  # some wire positions repeated: zero-length intervals
        s = synth.tiny(90, 3, 23, 61, seed=210, n_src=6, dark=100.0, render_now=False)
        _tilted_detector(s, [200.0, 8.0, 28.0])
        c = s.wire.centers
        idx = np.sort(np.concatenate([np.arange(c.shape[0]), [0, 5, 5, 11, c.shape[0] - 1]]))
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(c[idx]))
    elif name == "tilted_near_repeated":  # wire positions a hair apart: steps of ~1e-7 bins
        s = synth.tiny(90, 3, 23, 61, seed=215, n_src=6, dark=100.0, render_now=False)
        _tilted_detector(s, [200.0, 8.0, 28.0])
        c = s.wire.centers
        idx = np.sort(np.concatenate([np.arange(c.shape[0]), [2, 9, 9, 16]]))
        c = c[idx].copy()
        # each repeat moved 1e-7 um further along the scan (y and z by 1e-7/sqrt(2))
        rep = np.concatenate([[False], idx[1:] == idx[:-1]])
        bump = np.cumsum(rep) * rep * (1e-7 / math.sqrt(2.0))
        c[:, 1] += bump
        c[:, 2] += bump
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(c))
    elif name == "tilted_decreasing_repeated":  # backwards, with zero-length steps
        s = synth.tiny(128, 3, 33, 101, seed=212, n_src=8, dark=100.0, render_now=False)
        _tilted_detector(s, [200.0, 0.0, -30.0])
        c = s.wire.centers[::-1]
        idx = np.sort(np.concatenate([np.arange(c.shape[0]), [0, 3, 3, 17, c.shape[0] - 1]]))
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(c[idx]))
    elif name == "pixel_table_mixed_directions":  # neighbouring shadows move opposite ways
        # a pixel more than the detector distance downstream of the wire sees
        # the wire's leading edge sweep the beam backwards: every other column
        # sits 700 mm downstream, so every wave holds lanes walking both ways
        s = synth.tiny(96, 3, 31, 181, seed=213, n_src=8, dark=100.0, render_now=False)
        x, y, z = s.detector.pixel_xyz_arrays()
        z = z + np.where(np.arange(96)[None, :] % 2 == 1, 700000.0, 0.0)
        d = s.detector
        s.detector = synth.Detector(d.nx, d.ny, d.origin, d.u, d.v,
                                    pixel_xyz=np.stack([x, y, z], -1))
        s.grid = synth.DepthGrid(181, -540.0 + 1.5, 3.0)
        s.name = name
        # the far pixels see no source occluded; counts drawn at random give
        # every pixel intensity differences to spread
        rng = np.random.default_rng(213)
        s.images = rng.integers(0, 4000, (31, 3, 96)).astype(np.uint16)
        return s
    elif name == "pixel_table_spread":  # one direction, shadows of a wave tens of bins apart
        s = synth.tiny(80, 3, 29, 121, seed=214, n_src=8, dark=100.0, render_now=False)
        x, y, z = s.detector.pixel_xyz_arrays()
        z = z + np.linspace(-100000.0, 100000.0, 80)[None, :]
        d = s.detector
        s.detector = synth.Detector(d.nx, d.ny, d.origin, d.u, d.v,
                                    pixel_xyz=np.stack([x, y, z], -1))
        s.grid = synth.DepthGrid(121, -100.0 + 0.5, 1.0)
        s.name = name
        synth.render(s)
        return s
    elif name == "tilted_partial_grid":  # grid narrower than the sweeps: both ends leave it
        s = synth.tiny(100, 3, 31, 25, seed=211, n_src=6, dark=100.0, render_now=False)
        _tilted_detector(s, [200.0, -6.0, 22.0])
        s.grid = synth.DepthGrid(25, -7.7, 0.6)
        s.name = name
        synth.render(s)
        return s
    elif name.startswith("trailing_") or name.startswith("both_"):
        edge, base = name.split("_", 1)
        s = make_case(base)
        s.wire.edge = synth.EDGE_TRAILING if edge == "trailing" else synth.EDGE_BOTH
        return s
    else:
        raise KeyError(name)
    if name not in ("tilted_coarse", "tilted_many_bins"):
        _cover(s)
    synth.render(s)
    return s


CASES = ["tilted_detector", "axis_xz", "axis_xy", "axis_oblique", "pixel_table_jitter",
         "tilted_non_monotone", "tilted_coarse", "tilted_decreasing", "tilted_many_bins",
         "tilted_repeated_steps", "tilted_near_repeated", "tilted_partial_grid",
         "tilted_decreasing_repeated",
         "pixel_table_mixed_directions", "pixel_table_spread",
         "trailing_tilted_detector",
         "trailing_axis_xz", "both_axis_xy", "both_tilted_non_monotone", "both_axis_oblique"]


@pytest.mark.parametrize("name", CASES)
def test_takes_per_pixel_path(dr, ctx, name):
    s = make_case(name)
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        assert dr.dr_geometry_path(g) == dr.DR_PATH_PIXELS
    finally:
        dr.dr_geometry_free(g)


@pytest.mark.parametrize("name", CASES)
def test_positions_bit_exact(dr, ctx, name):
    s = make_case(name)
    nx, ny = s.detector.nx, s.detector.ny
    rng = np.random.default_rng(2)
    pix = np.unique(np.concatenate([[0, nx - 1, nx * ny - 1], rng.integers(0, nx * ny, 64)]))
    edges = {synth.EDGE_LEADING: [0], synth.EDGE_TRAILING: [1], synth.EDGE_BOTH: [0, 1]}
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        for side in edges[s.wire.edge]:
            w = synth.Wire(s.wire.radius, s.wire.centers, axis=s.wire.axis, edge=side)
            ref_scan = synth.Scan(s.name, s.detector, w, s.grid, s.sources, s.dark, s.noise,
                                  s.seed)
            _, bins_ref, u_ref = oracle.reconstruct_pixels(ref_scan, pix, want_bins=True,
                                                           want_u=True)
            bins, u = dr.dr_debug_plan(g, pix, s.wire.n_steps, edge=side)
            assert np.array_equal(bins, bins_ref), side
            assert np.array_equal(u.view(np.int64), u_ref.view(np.int64)), side
    finally:
        dr.dr_geometry_free(g)


@pytest.mark.parametrize("name", CASES)
def test_f64_instance_bit_exact(dr, ctx, name):
    s = make_case(name)
    out_ref, tot_ref, _ = oracle.reconstruct(s)
    out, tot = run_f64(dr, ctx, s)
    assert np.array_equal(out.view(np.int64), out_ref.view(np.int64)), \
        float(np.abs(out - out_ref).max())
    scale = np.abs(np.diff(s.images.astype(np.float64), axis=0)).sum()
    assert np.all(np.abs(tot - tot_ref) <= 1e-12 * max(scale, 1.0))


@pytest.mark.parametrize("name", CASES)
def test_f32_within_tolerance(dr, ctx, name):
    s = make_case(name)
    out_ref, tot_ref, _ = oracle.reconstruct(s)
    out, tot = run_f32(dr, ctx, s)
    assert_f32_close(out, out_ref, s.images)
    assert_totals_close(tot, tot_ref, s.images)


@pytest.mark.parametrize("name", ["tilted_detector", "both_axis_oblique"])
def test_slab_streaming_matches_device(dr, ctx, monkeypatch, name):
    s = make_case(name)
    dev, tot_d = run_f32(dr, ctx, s)
    for rows in ("1", "3", "64"):
        monkeypatch.setenv("DR_SLAB_ROWS", rows)
        host, tot_h = run_f32(dr, ctx, s, on_device=False)
        assert np.array_equal(host, dev), rows
        assert np.allclose(tot_h, tot_d, rtol=0, atol=1e-5 * max(1.0, np.abs(tot_d).max()))


@pytest.mark.parametrize("name", ["tilted_detector", "axis_oblique", "tilted_repeated_steps",
                                  "tilted_near_repeated"])
def test_fast_position_margin(dr, ctx, name):
    """The per-pixel path takes the shorter FP64 form of the positions (with
    exact bins) where the geometry's margin is small, the form's largest
    error (found at init over every pixel and step) is below half of it and
    every non-zero step is at least 2^28 times that error long; exact repeats
    of a wire position (zero steps) keep it, positions a hair apart (steps of
    ~1e-7 bins) make every position exact.  The other tests hold both forms
    to the oracle."""
    s = make_case(name)
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        m, err = dr.dr_geometry_position_margin(g)
        if name == "tilted_near_repeated":
            assert m >= 1.0, m
        else:
            assert 0.0 < m < 2.0 ** -12, m
        # the two forms evaluated at every pixel and step: the bound holds
        # with room (it is taken 2^9 above the errors it models)
        assert 0.0 <= err <= m / 64.0, (err, m)
    finally:
        dr.dr_geometry_free(g)
    flat = synth.tiny(40, 6, 21, 51, seed=209, n_src=5, dark=100.0)
    g = dr.dr_geometry_init(ctx, flat.detector, flat.wire, flat.grid)
    try:
        assert dr.dr_geometry_position_margin(g) == (0.0, 0.0)  # per-row path
    finally:
        dr.dr_geometry_free(g)


def test_row_uniform_geometries_keep_row_path(dr, ctx):
    """A flat detector with columns along the wire axis, and an explicit table
    whose rows repeat one (y, z), keep the per-row tables."""
    s = synth.tiny(40, 6, 21, 51, seed=209, n_src=5, dark=100.0)
    x, y, z = s.detector.pixel_xyz_arrays()
    d = s.detector
    table = synth.Detector(d.nx, d.ny, d.origin, d.u, d.v,
                           pixel_xyz=np.stack([x + 3.0, y, z], -1))
    for det in (d, table):
        g = dr.dr_geometry_init(ctx, det, s.wire, s.grid)
        try:
            assert dr.dr_geometry_path(g) == dr.DR_PATH_ROWS
        finally:
            dr.dr_geometry_free(g)


def test_per_pixel_entry_points(dr, ctx):
    """A per-pixel geometry has a single launch shape."""
    import torch
    s = make_case("tilted_detector")
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        img = torch.zeros(s.images.shape, dtype=torch.int16, device="cuda")
        out = torch.zeros((s.grid.n_bins, s.detector.ny, s.detector.nx), device="cuda")
        assert dr.dr_autotune(g, img, out)[:3] == (1, 4, 8)
        with pytest.raises(dr.DRError) as e:
            dr.dr_set_tile(g, (2, 4, 16))
        assert e.value.code == dr.DR_E_UNSUPPORTED
        dr.dr_set_tile(g, None)
        torch.cuda.synchronize()
    finally:
        dr.dr_geometry_free(g)


def test_grid_too_fine_for_the_sweep_refused(dr, ctx):
    """Per-pixel positions are bin indices in int32 arithmetic: a grid so fine
    that an edge position lies 2^30 bins or more from its first bin is refused
    when the geometry is built."""
    s = make_case("tilted_detector")
    fine = synth.DepthGrid(101, -5.0e-7, 1.0e-8)  # edge positions up to ~1.7e9 bins of 0.01 pm
    with pytest.raises(dr.DRError) as e:
        dr.dr_geometry_init(ctx, s.detector, s.wire, fine)
    assert e.value.code == dr.DR_E_INVAL and "2^30" in str(e.value)


@pytest.mark.parametrize("name", ["tilted_detector", "tilted_decreasing", "both_axis_oblique",
                                  "pixel_table_spread"])
def test_totals_repeatable(dr, ctx, name):
    """Totals do not depend on the order in which the hardware runs the
    workgroups: the FP32 kernel sums each wave's closed bins through its LDS
    ring in a fixed tree and adds the wave rows in order, and the FP64
    instance sums its finished output in a fixed order.  Five runs each must
    agree bit for bit (FP64 on every case; FP32 where every close falls in the
    ring, i.e. all but the case whose shadows lie ~90 bins apart in a wave)."""
    s = make_case(name)
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        t64 = [run_f64(dr, ctx, s)[1] for _ in range(5)]
        assert all(np.array_equal(t.view(np.int64), t64[0].view(np.int64)) for t in t64)
        if name != "pixel_table_spread":
            t32 = [run_f32(dr, ctx, s, geom=g)[1] for _ in range(5)]
            assert all(np.array_equal(t.view(np.int32), t32[0].view(np.int32)) for t in t32)
    finally:
        dr.dr_geometry_free(g)


def test_positions_on_bin_edges(dr, ctx):
    """Edge positions that land exactly on bin edges.  With a 1 um grid whose
    lower edge e0 is d - m for the exact depth d of one pixel at one step
    (d - m is exact by Sterbenz's lemma for |d| >= 2 and m = floor(d)), that
    position is exactly an integer in bin units.  The kernel's fast position
    there lies within its error bound of the integer and must fall back to
    the exact one: bins, FP64 output and FP32 output against the oracle as
    everywhere."""
    base = make_case("tilted_detector")
    grid0 = synth.DepthGrid(base.grid.n_bins, 0.5, 1.0)  # e0 = 0: u = d exactly
    probe = synth.Scan(base.name, base.detector, base.wire, grid0, base.sources, base.dark,
                       base.noise, base.seed)
    nx = base.detector.nx
    pix = np.arange(nx, 2 * nx, 37, dtype=np.int64)
    _, _, u = oracle.reconstruct_pixels(probe, pix, want_bins=False, want_u=True)
    ok = np.argwhere(np.abs(u) >= 2.0)
    assert ok.shape[0] > 0
    i, k = ok[ok.shape[0] // 2]
    d = float(u[i, k])
    m = math.floor(d)
    e0 = d - m
    assert e0 + m == d and (e0 + 0.5) - 0.5 == e0
    lo = math.floor(float(u.min())) - m - 4
    B = int(math.ceil(float(u.max())) - m + 4 - lo)
    # bin b of the new grid covers [e0 + (b + lo) um, ...): first centre e0 + lo + 0.5
    s = synth.Scan("bin_edges", base.detector, base.wire,
                   synth.DepthGrid(B, (e0 + lo) + 0.5, 1.0), base.sources, base.dark, base.noise,
                   base.seed)
    s.images = base.images
    _, bins_ref, u_ref = oracle.reconstruct_pixels(s, pix, want_bins=True, want_u=True)
    assert float(u_ref[i, k]) == float(m - lo)  # exactly on a bin edge
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        bins, upos = dr.dr_debug_plan(g, pix, s.wire.n_steps)
        assert np.array_equal(bins, bins_ref)
        assert np.array_equal(upos.view(np.int64), u_ref.view(np.int64))
    finally:
        dr.dr_geometry_free(g)
    out_ref, tot_ref, _ = oracle.reconstruct(s)
    out64, _ = run_f64(dr, ctx, s)
    assert np.array_equal(out64.view(np.int64), out_ref.view(np.int64))
    out, tot = run_f32(dr, ctx, s)
    assert_f32_close(out, out_ref, s.images)
    assert_totals_close(tot, tot_ref, s.images)
