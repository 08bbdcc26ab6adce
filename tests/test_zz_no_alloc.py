"""dr_reconstruct_noalloc (scratch from the library's fixed device array)
against dr_reconstruct (scratch from the geometry's own buffers), through the
C ABI: two calls in a row on the same GPU, the second on a smaller scan, each
bitwise equal to dr_reconstruct and within 1e-5 * sum_k |dI_k| of the oracle
on sampled pixels; a scan whose totals need more scratch than the array holds
is refused before any device work.  Needs an MI355X."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, abs_diff_scale, dev_images

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


def both_ways(dr, ctx, scan, n_sample, seed):
    """(noalloc out, noalloc totals) after checking them against dr_reconstruct
    and sampled pixels against the oracle."""
    import torch
    B, ny, nx = scan.grid.n_bins, scan.detector.ny, scan.detector.nx
    g = dr.dr_geometry_init(ctx, scan.detector, scan.wire, scan.grid)
    stream = torch.cuda.current_stream()
    try:
        img = dev_images(scan.images)
        ref = torch.full((B, ny, nx), float("nan"), device="cuda")
        tref = torch.full((B,), float("nan"), device="cuda")
        dr.dr_reconstruct(g, img, True, ref, tref, stream)
        out = torch.full((B, ny, nx), float("nan"), device="cuda")
        tot = torch.full((B,), float("nan"), device="cuda")
        # twice into the same buffers: the second run must not see the first's scratch
        for _ in range(2):
            dr.dr_reconstruct_noalloc(g, img, out, tot, stream)
        out_nt = torch.full((B, ny, nx), float("nan"), device="cuda")
        dr.dr_reconstruct_noalloc(g, img, out_nt, None, stream)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), scan.name
        assert torch.equal(out_nt.view(torch.int32), ref.view(torch.int32)), scan.name
        assert torch.equal(tot.view(torch.int32), tref.view(torch.int32)), scan.name
        rng = np.random.default_rng(seed)
        pix = np.unique(np.concatenate([[0, nx * ny - 1], rng.integers(0, nx * ny, n_sample)]))
        want, _, _ = oracle.reconstruct_pixels(scan, pix, want_bins=False)
        got = out.view(B, -1)[:, torch.from_numpy(pix).cuda()].T.cpu().numpy().astype(np.float64)
        scale = abs_diff_scale(scan.images).reshape(-1)[pix]
        err = np.abs(got - want)
        assert np.all(err <= REL_TOL * scale[:, None]), float(
            (err / np.maximum(scale[:, None], 1e-300)).max())
        return out, tot
    finally:
        dr.dr_geometry_free(g)


def test_noalloc_two_calls_second_smaller(dr, ctx):
    import torch
    big = synth.config2()
    small = synth.config1()
    both_ways(dr, ctx, big, 1500, 61)
    both_ways(dr, ctx, small, 600, 62)
    # the small scan's totals against the oracle's (whole scan)
    g = dr.dr_geometry_init(ctx, small.detector, small.wire, small.grid)
    try:
        img = dev_images(small.images)
        out = torch.empty((small.grid.n_bins, small.detector.ny, small.detector.nx),
                          device="cuda")
        tot = torch.full((small.grid.n_bins,), float("nan"), device="cuda")
        dr.dr_reconstruct_noalloc(g, img, out, tot, torch.cuda.current_stream())
        torch.cuda.synchronize()
        ref, tref, _ = oracle.reconstruct(small)
        scale = abs_diff_scale(small.images)
        assert np.all(np.abs(out.cpu().numpy().astype(np.float64) - ref) <= REL_TOL * scale[None])
        assert np.all(np.abs(tot.cpu().numpy().astype(np.float64) - tref) <=
                      REL_TOL * scale.sum())
    finally:
        dr.dr_geometry_free(g)


def test_noalloc_refuses_oversized_scratch(dr, ctx):
    """Two edges over 2048^2 pixels and 1500 bins need at least
    2 passes x 8 partial rows per detector row x 2048 rows x 1500 bins x 4 B
    = 197 MB of partial totals, more than the 128 MiB array: refused, and the
    output is left untouched (the buffers are full-size, so nothing could be
    written out of bounds even if the check were missing)."""
    import torch
    nx = ny = 2048
    B, N = 1500, 3
    det = synth.flat_detector(nx, ny, 200.0)
    wire = synth.wire_scan(N, 0.5)
    wire.edge = dr.DR_EDGE_BOTH
    grid = synth.centered_grid(B, 0.5)
    g = dr.dr_geometry_init(ctx, det, wire, grid)
    try:
        img = torch.zeros((N, ny, nx), dtype=torch.int16, device="cuda")
        out = torch.full((B, ny, nx), 7.0, device="cuda")
        tot = torch.full((B,), 7.0, device="cuda")
        with pytest.raises(dr.DRError) as e:
            dr.dr_reconstruct_noalloc(g, img, out, tot, torch.cuda.current_stream())
        assert e.value.code == dr.DR_E_INVAL and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert bool((tot == 7.0).all()) and bool((out[:, :8] == 7.0).all())
    finally:
        dr.dr_geometry_free(g)
        torch.cuda.empty_cache()


def test_noalloc_full_frame(dr, ctx):
    """The largest scan the fixed array serves: 2048^2 px, 1001 steps, 1001
    bins with totals (125.6 MiB of partial rows at the autotuned (2, 4, 16)
    shape), bitwise equal to dr_reconstruct, then a smaller scan again."""
    import torch
    s = synth.config3()
    B, ny, nx = s.grid.n_bins, s.detector.ny, s.detector.nx
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    stream = torch.cuda.current_stream()
    try:
        img = dev_images(s.images)
        s.images = None
        dr.dr_set_tile(g, (2, 4, 16))
        ref = torch.empty((B, ny, nx), device="cuda")
        tref = torch.empty((B,), device="cuda")
        dr.dr_reconstruct(g, img, True, ref, tref, stream)
        out = torch.full((B, ny, nx), float("nan"), device="cuda")
        tot = torch.full((B,), float("nan"), device="cuda")
        dr.dr_reconstruct_noalloc(g, img, out, tot, stream)
        torch.cuda.synchronize()
        for r0 in range(0, ny, 64):
            assert torch.equal(out[:, r0:r0 + 64].view(torch.int32),
                               ref[:, r0:r0 + 64].view(torch.int32)), r0
        assert torch.equal(tot.view(torch.int32), tref.view(torch.int32))
        del img, ref, out
    finally:
        dr.dr_geometry_free(g)
        torch.cuda.empty_cache()
    both_ways(dr, ctx, synth.config1(), 300, 63)


def _with_weights(s, seed):
    w = np.random.default_rng(seed).uniform(0.5, 2.0, s.wire.n_steps)
    s.wire = synth.Wire(s.wire.radius, s.wire.centers, axis=s.wire.axis, edge=s.wire.edge,
                        weights=w)
    return s


def _tilted(s, u):
    d = s.detector
    s.detector = synth.Detector(d.nx, d.ny, d.origin, np.asarray(u, dtype=np.float64), d.v)
    synth.render(s)
    return s


def _every_path_case(name):
    if name == "rows_both_edges":
        s = synth.tiny(160, 5, 33, 141, seed=701, n_src=10, dark=100.0)
        s.grid = synth.DepthGrid(141, -71.5 + 0.35, 0.7)
        s.wire.edge = synth.EDGE_BOTH
    elif name == "rows_non_monotone":  # the generic (read-modify-write) row body
        s = synth.tiny(96, 6, 31, 81, seed=702, n_src=8, dark=100.0)
        c = s.wire.centers
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(np.concatenate([c, c[::-1][1:]])))
        synth.render(s)
    elif name == "rows_weighted":
        s = _with_weights(synth.tiny(300, 7, 37, 61, seed=703, n_src=12, dark=100.0), 704)
    elif name == "pixels_both_edges":  # per-pixel kernel, two passes
        s = _tilted(synth.tiny(300, 4, 31, 81, seed=705, n_src=10, dark=100.0,
                               render_now=False), [200.0, 15.0, 35.0])
        s.grid = synth.DepthGrid(81, -72.0 + 0.6, 1.2)
        s.wire.edge = synth.EDGE_BOTH
    elif name == "pixels_many_bins":  # partial totals beyond the kernel's LDS ring
        s = _tilted(synth.tiny(40, 2, 21, 20000, seed=706, n_src=4, dark=100.0, width=0.002,
                               render_now=False), [200.0, 0.0, 10.0])
    elif name == "pixels_weighted":
        s = _with_weights(_tilted(synth.tiny(300, 4, 31, 81, seed=707, n_src=10, dark=100.0,
                                             render_now=False), [200.0, 15.0, 35.0]), 708)
    else:
        raise KeyError(name)
    s.name = name
    return s


@pytest.mark.parametrize("name", ["rows_both_edges", "rows_non_monotone", "rows_weighted",
                                  "pixels_both_edges", "pixels_many_bins", "pixels_weighted"])
def test_noalloc_every_path(dr, ctx, name):
    """Every kernel path that writes scratch (two-edge passes, the generic row
    body, step weights, the per-pixel kernel, and its totals summed in place
    when the bins outgrow its LDS): bitwise equal to dr_reconstruct, with and
    without totals, twice in a row into the same buffers."""
    import torch
    s = _every_path_case(name)
    B, ny, nx = s.grid.n_bins, s.detector.ny, s.detector.nx
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    stream = torch.cuda.current_stream()
    try:
        img = dev_images(s.images)
        ref = torch.full((B, ny, nx), float("nan"), device="cuda")
        tref = torch.full((B,), float("nan"), device="cuda")
        dr.dr_reconstruct(g, img, True, ref, tref, stream)
        out = torch.full((B, ny, nx), float("nan"), device="cuda")
        tot = torch.full((B,), float("nan"), device="cuda")
        for _ in range(2):
            dr.dr_reconstruct_noalloc(g, img, out, tot, stream)
        out_nt = torch.full((B, ny, nx), float("nan"), device="cuda")
        dr.dr_reconstruct_noalloc(g, img, out_nt, None, stream)
        torch.cuda.synchronize()
        assert not bool(torch.isnan(ref).any()) and not bool(torch.isnan(tref).any())
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), name
        assert torch.equal(out_nt.view(torch.int32), ref.view(torch.int32)), name
        assert torch.equal(tot.view(torch.int32), tref.view(torch.int32)), name
    finally:
        dr.dr_geometry_free(g)
