"""HIP path against the FP64 oracle, through the C ABI (needs an MI355X).

* bin indices floor(u_k) and positions u_k: bit-exact;
* the FP64-accumulation instance: bit-exact output;
* the FP32 path: |gpu - oracle| <= 1e-5 * sum_k |I_k - I_{k+1}| per pixel and
  bin; totals within 1e-5 of the summed scale;
* launch shapes, slab streaming and the paper's row-slab example: bitwise
  equal to the plain device run.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (assert_f32_close, assert_totals_close, dev_images, run_f32, run_f64)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def _rewire(s, centers):
    s.wire = synth.Wire(radius=s.wire.radius, centers=np.ascontiguousarray(centers))
    synth.render(s)
    return s


def make_case(name):
    if name == "config1":
        return synth.config1()
    if name == "ragged_301x7":  # odd width: one pixel per lane, ragged last tile
        return synth.tiny(301, 7, 37, 45, seed=101, n_src=12, dark=100.0)
    if name == "wide_2500x5":   # several tiles per row and a ragged tail
        return synth.tiny(2500, 5, 29, 61, seed=102, n_src=40, dark=100.0, pitch=150.0)
    if name == "long_1500_steps":  # more intervals than one LDS plan chunk
        return synth.tiny(64, 3, 1500, 900, seed=103, n_src=6, dark=100.0, step=0.5, width=0.5)
    if name == "decreasing":    # wire scanned backwards: -z leading edge, bins visited downwards
        s = synth.tiny(128, 9, 41, 101, seed=104, n_src=10, dark=100.0)
        return _rewire(s, s.wire.centers[::-1])
    if name == "non_monotone":  # forward then back: generic read-modify-write path
        s = synth.tiny(96, 6, 31, 81, seed=105, n_src=8, dark=100.0)
        c = s.wire.centers
        return _rewire(s, np.concatenate([c, c[::-1][1:]], axis=0))
    if name == "narrow_grid":   # most of every sweep falls outside the grid
        return synth.tiny(64, 8, 41, 5, seed=106, n_src=10, dark=100.0)
    if name == "coarse_steps":  # each interval spans many bins
        return synth.tiny(80, 4, 12, 300, seed=107, n_src=6, dark=100.0, step=4.0, width=0.1)
    if name == "degenerate_1x1":
        return synth.tiny(1, 1, 2, 1, seed=108, n_src=1, dark=100.0, sigma=0.0, zlo=-0.3,
                          zhi=0.3)
    if name == "pixel_table":   # explicit per-pixel centres (row-uniform)
        s = synth.tiny(40, 6, 21, 51, seed=109, n_src=5, dark=100.0)
        py, pz = s.detector.pixel_yz()
        xyz = np.zeros((6, 40, 3))
        xyz[..., 0] = np.arange(40)[None, :] * 200.0
        xyz[..., 1] = py
        xyz[..., 2] = pz
        s.detector = synth.Detector(40, 6, s.detector.origin, s.detector.u, s.detector.v,
                                    pixel_xyz=xyz)
        return s
    if name == "many_bins":      # 20000 bins: partial-total windows and zero fill at scale
        return synth.tiny(64, 3, 41, 20000, seed=114, n_src=6, dark=100.0, width=0.002)
    if name == "wide_8191x2":    # long odd row: many tiles, ragged tail, one pixel per lane
        return synth.tiny(8191, 2, 25, 61, seed=115, n_src=30, dark=100.0, pitch=50.0)
    if name == "single_row":
        return synth.tiny(700, 1, 33, 81, seed=116, n_src=6, dark=100.0)
    if name.startswith("trailing_") or name.startswith("both_"):
        edge, base = name.split("_", 1)
        s = make_case(base)
        if base == "config1":
            s.grid = synth.centered_grid(201, 1.0)  # room for the trailing sweep
        s.wire.edge = synth.EDGE_TRAILING if edge == "trailing" else synth.EDGE_BOTH
        return s
    raise KeyError(name)


CASES = ["config1", "ragged_301x7", "wide_2500x5", "long_1500_steps", "decreasing",
         "non_monotone", "narrow_grid", "coarse_steps", "degenerate_1x1", "pixel_table",
         "trailing_config1", "trailing_decreasing", "both_config1", "both_ragged_301x7",
         "both_decreasing", "both_non_monotone", "both_long_1500_steps", "many_bins",
         "wide_8191x2", "single_row", "both_many_bins"]


@pytest.mark.parametrize("name", CASES)
def test_positions_bit_exact(dr, ctx, name):
    s = make_case(name)
    nx, ny = s.detector.nx, s.detector.ny
    rng = np.random.default_rng(1)
    pix = np.unique(np.concatenate([[0, nx * ny - 1], rng.integers(0, nx * ny, 64)]))
    edges = {synth.EDGE_LEADING: [0], synth.EDGE_TRAILING: [1], synth.EDGE_BOTH: [0, 1]}
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        for side in edges[s.wire.edge]:
            ref_scan = synth.Scan(s.name, s.detector, synth.Wire(s.wire.radius, s.wire.centers,
                                                                  edge=side), s.grid,
                                  s.sources, s.dark, s.noise, s.seed)
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


def test_launch_shapes_bitwise_equal(dr, ctx):
    s = make_case("wide_2500x5")
    ref, tot_ref, _ = oracle.reconstruct(s)
    base, _ = run_f32(dr, ctx, s, tile=(1, 4, 4))
    for ppl in (1, 2, 4):  # 2500 is not a multiple of 8
        for waves in (2, 4):
            for pf in (4, 8):
                out, tot = run_f32(dr, ctx, s, tile=(ppl, waves, pf))
                assert np.array_equal(out, base), (ppl, waves, pf)
                assert_totals_close(tot, tot_ref, s.images)
    s8 = synth.tiny(1024, 3, 23, 41, seed=110, n_src=8, dark=100.0)
    b8, _ = run_f32(dr, ctx, s8, tile=(1, 2, 4))
    for waves in (2, 4):
        for pf in (4, 8):
            assert np.array_equal(run_f32(dr, ctx, s8, tile=(8, waves, pf))[0], b8)


def test_slab_streaming_matches_device(dr, ctx, monkeypatch):
    s = synth.tiny(256, 37, 33, 61, seed=111, n_src=10, dark=100.0)
    dev, tot_d = run_f32(dr, ctx, s)
    for rows in ("1", "5", "37", "64"):
        monkeypatch.setenv("DR_SLAB_ROWS", rows)
        host, tot_h = run_f32(dr, ctx, s, on_device=False)
        assert np.array_equal(host, dev), rows
        assert np.array_equal(tot_h, tot_d), rows


def test_paper_worked_example_row_slabs(dr, ctx, monkeypatch):
    """4 images x 6 rows x 9 columns in 2-row passes equals one pass."""
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    s = synth.tiny(ex["n_cols"], ex["n_rows"], ex["n_images"], 7, seed=3, pitch=2000.0,
                   step=2.0, width=1.0, n_src=3, dark=20.0)
    one, _ = run_f32(dr, ctx, s)
    monkeypatch.setenv("DR_SLAB_ROWS", str(ex["rows_per_pass"]))
    passes, _ = run_f32(dr, ctx, s, on_device=False)
    assert np.array_equal(one, passes)
    ref, _, _ = oracle.reconstruct(s)
    assert_f32_close(passes, ref, s.images)


def test_geometry_errors(dr, ctx):
    s = synth.tiny(8, 4, 5, 9, seed=112, n_src=1)
    bad = synth.Wire(radius=s.wire.radius, centers=s.wire.centers.copy())
    bad.centers[:, 1] = -5.0  # wire below the beam
    with pytest.raises(dr.DRError) as e:
        dr.dr_geometry_init(ctx, s.detector, bad, s.grid)
    assert e.value.code == dr.DR_E_INVAL
    inside = synth.Wire(radius=1e6, centers=s.wire.centers.copy())  # pixels inside the wire
    with pytest.raises(dr.DRError) as e:
        dr.dr_geometry_init(ctx, s.detector, inside, s.grid)
    assert e.value.code == dr.DR_E_INVAL
    tilted = synth.Detector(8, 4, s.detector.origin, np.array([200.0, 0.0, 1.0]), s.detector.v)
    g = dr.dr_geometry_init(ctx, tilted, s.wire, s.grid)  # per-pixel path, accepted
    assert dr.dr_geometry_path(g) == dr.DR_PATH_PIXELS
    dr.dr_geometry_free(g)
    for axis in ([0.0, 0.0, 1.0], [0.0, 0.0, -2.0], [0.0, 0.0, 0.0]):  # along the beam, zero
        w_axis = synth.Wire(radius=26.0, centers=s.wire.centers, axis=np.array(axis))
        with pytest.raises(dr.DRError) as e:
            dr.dr_geometry_init(ctx, s.detector, w_axis, s.grid)
        assert e.value.code == dr.DR_E_INVAL, axis
    # axis along y: eta = -x, negative for half the detector (wire not between)
    w_axis = synth.Wire(radius=26.0, centers=s.wire.centers, axis=np.array([0.0, 1.0, 0.0]))
    with pytest.raises(dr.DRError) as e:
        dr.dr_geometry_init(ctx, s.detector, w_axis, s.grid)
    assert e.value.code == dr.DR_E_INVAL


def test_all_zero_outside_sweep(dr, ctx):
    """Bins the leading edge never reaches are written as exact zeros."""
    s = synth.tiny(64, 4, 9, 400, seed=113, n_src=3, dark=100.0)
    out, _ = run_f32(dr, ctx, s)
    pix = np.arange(64 * 4)
    _, bins, _ = oracle.reconstruct_pixels(s, pix, want_bins=True)
    b = np.arange(400)[:, None]
    outside = (b < bins.min(1)[None, :]) | (b > bins.max(1)[None, :])
    flat = out.reshape(400, -1)
    assert outside.any() and np.all(flat[outside] == 0.0)
