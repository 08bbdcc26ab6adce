"""Full-size workloads in the launch configuration the benchmark times
(autotuned shape, images resident in HBM), needs an MI355X.

* 1024^2 px x 401 steps x 501 bins: the whole output against the oracle;
* 2048^2 px x 1001 steps x 1001 bins: sampled pixels against the oracle
  (FP32 tolerance, bit-exact positions, bit-exact FP64 instance), intensity
  conservation for every pixel whose sweep lies inside the grid, and the
  totals against an FP64 sum of the output.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, assert_f32_close, assert_totals_close

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


def _render_pinned(scan):
    import torch
    N, ny, nx = scan.wire.n_steps, scan.detector.ny, scan.detector.nx
    host = torch.empty((N, ny, nx), dtype=torch.int16, pin_memory=True)
    synth.render(scan, out=host.numpy().view(np.uint16))
    return host


def _run_like_bench(dr, ctx, scan, host):
    import torch
    det, grid = scan.detector, scan.grid
    dev = host.to("cuda")
    out = torch.full((grid.n_bins, det.ny, det.nx), float("nan"), device="cuda")
    tot = torch.full((grid.n_bins,), float("nan"), device="cuda")
    g = dr.dr_geometry_init(ctx, det, scan.wire, grid)
    dr.dr_autotune(g, dev, out)
    out.fill_(float("nan"))
    dr.dr_reconstruct(g, dev, True, out, tot, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return g, dev, out, tot


def _sample_pixels(nx, ny, n, seed):
    rng = np.random.default_rng(seed)
    edge = [0, nx - 1, (ny - 1) * nx, ny * nx - 1]
    rows = np.array([0, ny // 2, ny - 1])
    line = (rows[:, None] * nx + np.arange(0, nx, max(1, nx // 64))[None, :]).ravel()
    return np.unique(np.concatenate([edge, line, rng.integers(0, nx * ny, n)]))


def test_config2_whole_output(dr, ctx):
    import torch
    s = synth.config2(render_now=False)
    host = _render_pinned(s)
    s.images = host.numpy().view(np.uint16)
    g, dev, out, tot = _run_like_bench(dr, ctx, s, host)
    try:
        ref, tref, _ = oracle.reconstruct(s)
        assert_f32_close(out.cpu().numpy(), ref, s.images)
        assert_totals_close(tot.cpu().numpy(), tref, s.images)
    finally:
        dr.dr_geometry_free(g)
        del dev, out
        torch.cuda.empty_cache()


def test_config3_sampled_and_invariants(dr, ctx):
    import torch
    s = synth.config3(render_now=False)
    host = _render_pinned(s)
    s.images = host.numpy().view(np.uint16)
    det, grid, N = s.detector, s.grid, s.wire.n_steps
    nx, ny, B = det.nx, det.ny, grid.n_bins
    g, dev, out, tot = _run_like_bench(dr, ctx, s, host)
    try:
        assert not torch.isnan(out).any().item(), "unwritten output elements"
        pix = _sample_pixels(nx, ny, 3000, 33)
        ref, bins_ref, u_ref = oracle.reconstruct_pixels(s, pix, want_bins=True, want_u=True)
        flat = out.view(B, -1)
        got = flat[:, torch.from_numpy(pix).to("cuda")].T.cpu().numpy().astype(np.float64)
        series = s.images.reshape(N, -1)[:, pix].T
        scale = np.abs(np.diff(series.astype(np.int64), axis=1)).sum(1).astype(np.float64)
        assert np.all(np.abs(got - ref) <= REL_TOL * scale[:, None])
        bins, u = dr.dr_debug_plan(g, pix, N)
        assert np.array_equal(bins, bins_ref)
        assert np.array_equal(u.view(np.int64), u_ref.view(np.int64))
        # FP64 instance: bit-exact on the sample
        out64 = torch.empty((B, ny, nx), dtype=torch.float64, device="cuda")
        dr.dr_reconstruct_f64(g, dev, out64, None, torch.cuda.current_stream())
        torch.cuda.synchronize()
        got64 = out64.view(B, -1)[:, torch.from_numpy(pix).to("cuda")].T.cpu().numpy()
        assert np.array_equal(got64.view(np.int64), ref.view(np.int64))
        del out64
        torch.cuda.empty_cache()
        # conservation: rows whose whole sweep lies inside the grid
        row_pix = np.arange(ny) * nx
        rb, _ = dr.dr_debug_plan(g, row_pix, N, want_u=False)
        inside = (rb.min(1) >= 0) & (rb.max(1) <= B - 1)
        assert inside.sum() > ny // 3
        tot64 = torch.zeros(B, dtype=torch.float64, device="cuda")
        total_scale = 0.0
        for r0 in range(0, ny, 128):
            img = dev[:, r0:r0 + 128, :].to(torch.int32) & 0xFFFF  # uint16 counts
            sc = (img[1:] - img[:-1]).abs().sum(0).to(torch.float64)
            total_scale += float(sc.sum())
            first_minus_last = (img[0] - img[N - 1]).to(torch.float64)
            del img
            blk = out[:, r0:r0 + 128, :].to(torch.float64)
            tot64 += blk.sum(dim=(1, 2))
            sums = blk.sum(0)
            del blk
            rows = torch.from_numpy(np.nonzero(inside[r0:r0 + 128])[0]).to("cuda")
            if rows.numel():
                d = (sums[rows] - first_minus_last[rows]).abs()
                assert bool((d <= REL_TOL * sc[rows] + 1e-6).all())
        assert float((tot.to(torch.float64) - tot64).abs().max()) <= REL_TOL * total_scale
        # pixel selection at full size: activities of the sample against the
        # oracle, the top-25% list obeys the rule, and its reconstruction from
        # full frames equals the dense output at the listed pixels bit for bit
        act = torch.empty(nx * ny, dtype=torch.int64, device="cuda")
        dr.dr_pixel_activity(g, dev, act, torch.cuda.current_stream())
        torch.cuda.synchronize()
        got_act = act[torch.from_numpy(pix).to("cuda")].cpu().numpy().view(np.uint64)
        assert np.array_equal(got_act, oracle.activity(np.ascontiguousarray(series.T)))
        k = nx * ny // 4
        lst = dr.dr_select_top(g, act, k)
        try:
            sel = torch.from_numpy(dr.dr_list_pixels(lst)).to("cuda")
            assert sel.numel() == k and bool((sel[1:] > sel[:-1]).all())
            chosen = torch.zeros(nx * ny, dtype=torch.bool, device="cuda")
            chosen[sel] = True
            thr = act[sel].min()
            assert bool((act[~chosen] <= thr).all()) and bool(chosen[act > thr].all())
            ties = torch.nonzero((act == thr) & ~chosen).flatten()
            if ties.numel():
                assert int(ties.min()) > int(sel[act[sel] == thr].max())
            outl = torch.empty((B, k), device="cuda")
            dr.dr_reconstruct_list(lst, dev, dr.DR_LAYOUT_FULL, True, outl, None,
                                   torch.cuda.current_stream())
            torch.cuda.synchronize()
            for c0 in range(0, k, 1 << 18):  # compare in column blocks
                cols = sel[c0:c0 + (1 << 18)]
                assert torch.equal(outl[:, c0:c0 + cols.numel()], out.view(B, -1)[:, cols])
            del outl, chosen
        finally:
            dr.dr_list_free(lst)
    finally:
        dr.dr_geometry_free(g)
        del dev, out
        torch.cuda.empty_cache()


def test_config3_per_pixel_path_sampled(dr, ctx):
    """2048^2 px x 1001 steps x 1001 bins with the detector's columns tilted
    out of the x axis: the per-pixel path, sampled pixels against the oracle
    (FP32 tolerance, bit-exact positions, bit-exact FP64 instance), and the
    fast positions' largest error, found at init, against their margin."""
    import torch
    s = synth.config3(render_now=False)
    d = s.detector
    s.detector = synth.Detector(d.nx, d.ny, d.origin, np.array([d.u[0], 0.0, 1.0]), d.v)
    host = _render_pinned(s)
    s.images = host.numpy().view(np.uint16)
    det, grid, N = s.detector, s.grid, s.wire.n_steps
    nx, ny, B = det.nx, det.ny, grid.n_bins
    g, dev, out, tot = _run_like_bench(dr, ctx, s, host)
    try:
        assert dr.dr_geometry_path(g) == dr.DR_PATH_PIXELS
        # fast positions in use, and their largest error over all 4.2e9
        # evaluations well inside the margin that certifies their floors
        m, err = dr.dr_geometry_position_margin(g)
        assert 0.0 < m < 2.0 ** -12 and err <= m / 64.0, (m, err)
        assert not torch.isnan(out).any().item(), "unwritten output elements"
        pix = _sample_pixels(nx, ny, 2000, 34)
        ref, bins_ref, u_ref = oracle.reconstruct_pixels(s, pix, want_bins=True, want_u=True)
        got = out.view(B, -1)[:, torch.from_numpy(pix).to("cuda")].T.cpu().numpy()
        series = s.images.reshape(N, -1)[:, pix].T
        scale = np.abs(np.diff(series.astype(np.int64), axis=1)).sum(1).astype(np.float64)
        assert np.all(np.abs(got.astype(np.float64) - ref) <= REL_TOL * scale[:, None])
        bins, u = dr.dr_debug_plan(g, pix, N)
        assert np.array_equal(bins, bins_ref)
        assert np.array_equal(u.view(np.int64), u_ref.view(np.int64))
        del out
        torch.cuda.empty_cache()
        out64 = torch.empty((B, ny, nx), dtype=torch.float64, device="cuda")
        dr.dr_reconstruct_f64(g, dev, out64, None, torch.cuda.current_stream())
        torch.cuda.synchronize()
        got64 = out64.view(B, -1)[:, torch.from_numpy(pix).to("cuda")].T.cpu().numpy()
        assert np.array_equal(got64.view(np.int64), ref.view(np.int64))
        del out64
    finally:
        dr.dr_geometry_free(g)
        del dev
        torch.cuda.empty_cache()
