"""Pixel activity, top-k selection and list reconstruction on the GPU (the
pixel-percentage experiment), needs an MI355X.

* activity: bit-exact (integers) against the oracle, vector and scalar loads;
* selection: the same list as the oracle's rule (ties to the lower index),
  including heavy ties and activities past 32 bits;
* list reconstruction: bitwise equal to the dense reconstruction at the listed
  pixels for every image layout (full frames, compact on the device, compact
  host stacks streamed in runs), FP64 instance bit-exact against the oracle,
  totals within tolerance; per-row and per-pixel paths, both edges.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_totals_close, dev_images, pinned_images, run_f32

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


def make_case(name):
    if name == "rows":          # per-row plans, ragged row width
        return synth.tiny(300, 7, 37, 61, seed=301, n_src=14, dark=100.0)
    if name == "rows_noise_free":  # many equal activities (dark 0, no noise)
        return synth.tiny(128, 6, 25, 51, seed=302, n_src=6, dark=0.0, noise=False)
    if name == "non_monotone":  # generic rows: read-modify-write path
        s = synth.tiny(96, 6, 31, 81, seed=303, n_src=8, dark=100.0)
        c = s.wire.centers
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(np.concatenate([c, c[::-1][1:]])))
        synth.render(s)
        return s
    if name == "both_rows":
        s = synth.tiny(200, 5, 33, 141, seed=304, n_src=10, dark=100.0)
        s.grid = synth.DepthGrid(141, -71.5 + 0.35, 0.7)
        s.wire.edge = synth.EDGE_BOTH
        return s
    if name == "tilted":        # per-pixel path
        s = synth.tiny(300, 4, 31, 81, seed=305, n_src=10, dark=100.0, render_now=False)
        d = s.detector
        s.detector = synth.Detector(d.nx, d.ny, d.origin, np.array([200.0, 15.0, 35.0]), d.v)
        synth.render(s)
        return s
    if name == "short_scan":    # fewer steps than the activity kernel's ring of loads
        return synth.tiny(64, 5, 9, 21, seed=308, n_src=4, dark=100.0)
    if name == "both_tilted":
        s = make_case("tilted")
        s.grid = synth.DepthGrid(81, -72.0 + 0.6, 1.2)
        s.wire.edge = synth.EDGE_BOTH
        return s
    raise KeyError(name)


CASES = ["rows", "rows_noise_free", "non_monotone", "both_rows", "tilted", "both_tilted"]


def _activity(dr, g, images, offset=0):
    import torch
    N, ny, nx = images.shape
    flat = torch.zeros(images.size + offset, dtype=torch.int16, device="cuda")
    flat[offset:] = torch.from_numpy(images.reshape(-1).view(np.int16)).to("cuda")
    act = torch.empty(nx * ny, dtype=torch.int64, device="cuda")
    dr.dr_pixel_activity(g, flat[offset:], act, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return act.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name", ["rows", "rows_noise_free", "tilted", "short_scan"])
def test_activity_exact(dr, ctx, name):
    s = make_case(name)
    ref = oracle.activity(s.images)
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        # 8-byte aligned (vector loads when nx*ny % 4 == 0: offsets 0, 4, 8) or not (1)
        for off in (0, 1, 4, 8):
            assert np.array_equal(_activity(dr, g, s.images, off), ref), off
    finally:
        dr.dr_geometry_free(g)


def _select(dr, g, act, k):
    import torch
    a = torch.from_numpy(np.ascontiguousarray(act).view(np.int64)).to("cuda")
    torch.cuda.synchronize()
    lst = dr.dr_select_top(g, a, k)
    try:
        return dr.dr_list_pixels(lst)
    finally:
        dr.dr_list_free(lst)


def test_select_top_matches_rule(dr, ctx):
    s = synth.tiny(64, 16, 5, 9, seed=306, n_src=2)
    npix = 64 * 16
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        rng = np.random.default_rng(306)
        acts = [rng.integers(0, 4, npix).astype(np.uint64),           # heavy ties
                rng.integers(0, 1 << 62, npix).astype(np.uint64),     # every radix digit
                np.zeros(npix, dtype=np.uint64),                      # all equal
                (rng.integers(0, 3, npix).astype(np.uint64) << np.uint64(40)) + np.uint64(7),
                # the top bit (keys compare unsigned; no digit is 0 in every key)
                (rng.integers(0, 2, npix).astype(np.uint64) << np.uint64(63))
                | rng.integers(0, 8, npix).astype(np.uint64)]
        for act in acts:
            for k in (0, 1, 2, 100, 341, 512, npix - 1, npix):
                got = _select(dr, g, act, k)
                assert np.array_equal(got, oracle.select_top(act, k)), k
        with pytest.raises(dr.DRError) as e:
            _select(dr, g, acts[0], npix + 1)
        assert e.value.code == dr.DR_E_INVAL
    finally:
        dr.dr_geometry_free(g)


def test_select_top_across_blocks(dr, ctx):
    """A detector of 300 x 47 pixels: the selection's key blocks (4096 keys)
    number three and a partial tail, so the scan carries between blocks, the
    padded last block and tie runs that straddle block boundaries are all
    exercised; k values cut tie runs in the middle of a block and at block
    edges."""
    s = synth.tiny(300, 47, 5, 9, seed=307, n_src=2)
    npix = 300 * 47
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        rng = np.random.default_rng(307)
        two = rng.integers(0, 2, npix).astype(np.uint64)
        steps = np.repeat(np.arange(7, dtype=np.uint64), npix // 7 + 1)[:npix][::-1].copy()
        acts = [rng.integers(0, 4, npix).astype(np.uint64),       # heavy ties
                np.full(npix, 9, dtype=np.uint64),                 # all equal
                two,                                               # one long tie run per value
                steps,                                             # runs ending inside blocks
                rng.integers(0, 1 << 62, npix).astype(np.uint64)]
        n_ones = int(two.sum())
        ks = sorted({0, 1, 4095, 4096, 4097, 8191, 8192, 12288, npix - 1, npix,
                     n_ones - 2500, n_ones - 1, n_ones, n_ones + 1, n_ones + 3000,
                     npix // 7 * 3 + 5})
        for a_i, act in enumerate(acts):
            for k in ks:
                got = _select(dr, g, act, k)
                assert np.array_equal(got, oracle.select_top(act, k)), (a_i, k)
    finally:
        dr.dr_geometry_free(g)


def _top_list(dr, g, s, frac):
    import torch
    npix = s.detector.nx * s.detector.ny
    act = _activity(dr, g, s.images)
    k = int(frac * npix)
    a = torch.from_numpy(act.view(np.int64)).to("cuda")
    torch.cuda.synchronize()
    lst = dr.dr_select_top(g, a, k)
    pix = dr.dr_list_pixels(lst)
    assert np.array_equal(pix, oracle.select_top(oracle.activity(s.images), k))
    return lst, pix


def _run_list(dr, lst, s, n, layout, on_device, images=None):
    import torch
    B = s.grid.n_bins
    out = torch.full((B, max(n, 1)), float("nan"), device="cuda")
    tot = torch.full((B,), float("nan"), device="cuda")
    im = s.images if images is None else images
    img = dev_images(im) if on_device else pinned_images(im)
    dr.dr_reconstruct_list(lst, img, layout, on_device, out, tot, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()[:, :n], tot.cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_list_equals_dense(dr, ctx, name, monkeypatch):
    s = make_case(name)
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        dense, _ = run_f32(dr, ctx, s, geom=g)
        flat = dense.reshape(s.grid.n_bins, -1)
        lst, pix = _top_list(dr, g, s, 0.3)
        try:
            n = pix.shape[0]
            N = s.wire.n_steps
            compact = np.ascontiguousarray(s.images.reshape(N, -1)[:, pix])
            ref_out, _, _ = oracle.reconstruct_pixels(s, pix)
            ref_tot = ref_out.sum(0)
            o1, t1 = _run_list(dr, lst, s, n, dr.DR_LAYOUT_FULL, True)
            assert np.array_equal(o1, flat[:, pix])
            assert_totals_close(t1, ref_tot, compact)
            o2, t2 = _run_list(dr, lst, s, n, dr.DR_LAYOUT_LIST, True, compact)
            assert np.array_equal(o2, o1)
            monkeypatch.setenv("DR_LIST_RUN_ENTRIES", "256")  # several host runs
            o3, t3 = _run_list(dr, lst, s, n, dr.DR_LAYOUT_LIST, False, compact)
            assert np.array_equal(o3, o1)
            assert_totals_close(t3, ref_tot, compact)
        finally:
            dr.dr_list_free(lst)
    finally:
        dr.dr_geometry_free(g)


@pytest.mark.parametrize("name", CASES)
def test_list_f64_bit_exact(dr, ctx, name):
    import torch
    s = make_case(name)
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        lst, pix = _top_list(dr, g, s, 0.5)
        try:
            n, B = pix.shape[0], s.grid.n_bins
            ref, _, _ = oracle.reconstruct_pixels(s, pix)
            out = torch.full((B, n), float("nan"), dtype=torch.float64, device="cuda")
            tot = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
            dr.dr_reconstruct_list_f64(lst, dev_images(s.images), dr.DR_LAYOUT_FULL, out, tot,
                                       torch.cuda.current_stream())
            torch.cuda.synchronize()
            got = out.cpu().numpy().T
            assert np.array_equal(got.view(np.int64), ref.view(np.int64))
            scale = np.abs(np.diff(s.images.astype(np.float64), axis=0)).sum()
            assert np.all(np.abs(tot.cpu().numpy() - ref.sum(0)) <= 1e-12 * max(scale, 1.0))
        finally:
            dr.dr_list_free(lst)
    finally:
        dr.dr_geometry_free(g)


def test_list_edge_cases(dr, ctx):
    import torch
    s = make_case("rows")
    npix = s.detector.nx * s.detector.ny
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        dense, _ = run_f32(dr, ctx, s, geom=g)
        # every pixel, from a host list: the dense output in flat order
        lst = dr.dr_list_create(g, np.arange(npix))
        try:
            o, _ = _run_list(dr, lst, s, npix, dr.DR_LAYOUT_FULL, True)
            assert np.array_equal(o, dense.reshape(s.grid.n_bins, -1))
            with pytest.raises(dr.DRError) as e:  # host images must be compact
                _run_list(dr, lst, s, npix, dr.DR_LAYOUT_FULL, False)
            assert e.value.code == dr.DR_E_INVAL
            with pytest.raises(dr.DRError) as e:  # the list keeps its geometry alive
                dr.dr_geometry_free(g)
            assert e.value.code == dr.DR_E_BUSY
        finally:
            dr.dr_list_free(lst)
        # an empty list: nothing written, totals zero
        lst = dr.dr_list_create(g, np.zeros(0, dtype=np.int64))
        try:
            assert dr.dr_list_size(lst) == 0
            out = torch.full((s.grid.n_bins, 1), 7.0, device="cuda")
            tot = torch.full((s.grid.n_bins,), 7.0, device="cuda")
            dr.dr_reconstruct_list(lst, dev_images(s.images), dr.DR_LAYOUT_FULL, True, out, tot,
                                   torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert bool((out == 7.0).all()) and bool((tot == 0.0).all())
        finally:
            dr.dr_list_free(lst)
        # a device list, single pixels at the row ends
        pix = np.array([0, 299, 300, npix - 1], dtype=np.int64)
        lst = dr.dr_list_create(g, torch.from_numpy(pix).to("cuda"), on_device=True)
        try:
            o, _ = _run_list(dr, lst, s, 4, dr.DR_LAYOUT_FULL, True)
            assert np.array_equal(o, dense.reshape(s.grid.n_bins, -1)[:, pix])
        finally:
            dr.dr_list_free(lst)
        for bad in ([3, 3], [5, 2], [-1], [npix]):
            with pytest.raises(dr.DRError) as e:
                dr.dr_list_create(g, np.array(bad, dtype=np.int64))
            assert e.value.code == dr.DR_E_INVAL, bad
    finally:
        dr.dr_geometry_free(g)
