"""Batched persistent launches and the serving scheduler (needs an MI355X).

Every pixel's bins are produced by the same tile code as the single-scan call,
so they must be bitwise equal alone, in a batch, in a replayed graph and in
the serving mix; totals (summed in a different grouping) agree within
1e-5 of the summed |dI| scale, and a sample of scans is checked against the
oracle.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (assert_f32_close, assert_totals_close, dev_images, pinned_images, run_f32)

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


def uneven_scans(seed, odd=False):
    """Scans of uneven ROI, step count and bin count (sub-windows of a 2048^2
    detector at 200 um, as in the batched workload, at test size)."""
    rng = np.random.default_rng(seed)
    scans = []
    for n in range(6):
        side = int(rng.choice([64, 96, 128]))
        nx = side + (1 if (odd and n == 2) else 0)
        N = int(rng.integers(31, 122))
        B = int(rng.integers(41, 162))
        i0, j0 = (int(x) for x in rng.integers(0, 2048 - side, 2))
        det = synth.flat_detector(nx, side, 200.0, full_nx=2048, full_ny=2048, i0=i0, j0=j0)
        wire = synth.wire_scan(N, 0.5)
        grid = synth.centered_grid(B, 0.5)
        half = 0.5 * min((N - 1) * 0.5 * 0.7, (B - 2) * 0.5)
        src = synth.draw_sources(rng, max(2, side * side // 800), nx, side, -half, half)
        s = synth.Scan(f"u{n}", det, wire, grid, src, dark=100.0, noise=True, seed=seed * 10 + n)
        synth.render(s)
        s.wire.edge = (synth.EDGE_LEADING, synth.EDGE_LEADING, synth.EDGE_BOTH,
                       synth.EDGE_LEADING, synth.EDGE_TRAILING, synth.EDGE_BOTH)[n]
        scans.append(s)
    return scans


def alone(dr, ctx, s):
    return run_f32(dr, ctx, s)


@pytest.mark.parametrize("odd", [False, True])
@pytest.mark.parametrize("flags", ["plain", "autotune+graph"])
def test_batch_matches_single_scans(dr, ctx, odd, flags):
    import torch
    scans = uneven_scans(7 if not odd else 8, odd=odd)
    singles = [alone(dr, ctx, s) for s in scans]
    geoms, imgs, outs, tots = [], [], [], []
    for s in scans:
        geoms.append(dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid))
        imgs.append(dev_images(s.images))
        outs.append(torch.full((s.grid.n_bins, s.detector.ny, s.detector.nx), float("nan"),
                               device="cuda"))
        tots.append(torch.full((s.grid.n_bins,), float("nan"), device="cuda"))
    f = 0 if flags == "plain" else (dr.DR_BATCH_AUTOTUNE | dr.DR_BATCH_GRAPH)
    torch.cuda.synchronize()
    b = dr.dr_batch_create(ctx, list(zip(geoms, imgs, outs, tots)), f)
    try:
        tile = dr.dr_batch_tile(b)
        if odd:
            assert tile[0] == 1
        stream = torch.cuda.current_stream()
        for rep in range(3):
            for o, t in zip(outs, tots):
                o.fill_(float("nan"))
                t.fill_(float("nan"))
            # unrelated eager work between replays
            junk = torch.randn(1 << 20, device="cuda").sum()
            dr.dr_batch_run(b, stream)
            torch.cuda.synchronize()
            del junk
            for s, (o1, t1), o, t in zip(scans, singles, outs, tots):
                o2 = o.cpu().numpy()
                assert np.array_equal(o2, o1), (rep, s.name)
                assert_totals_close(t.cpu().numpy(), t1.astype(np.float64), s.images)
    finally:
        dr.dr_batch_free(b)
        for g in geoms:
            dr.dr_geometry_free(g)
    for s in (scans[0], scans[2], scans[4]):  # leading, both, trailing
        ref, tref, _ = oracle.reconstruct(s)
        assert_f32_close(singles[scans.index(s)][0], ref, s.images)
        assert_totals_close(singles[scans.index(s)][1], tref, s.images)


def _serve(dr, ctx, scans, host_mask, wait_mode="poll"):
    import torch
    geoms = [dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid) for s in scans]
    outs = [torch.full((s.grid.n_bins, s.detector.ny, s.detector.nx), float("nan"),
                       device="cuda") for s in scans]
    tots = [torch.full((s.grid.n_bins,), float("nan"), device="cuda") for s in scans]
    imgs = [pinned_images(s.images) if h else dev_images(s.images) for s, h in zip(scans, host_mask)]
    torch.cuda.synchronize()
    tickets = [dr.dr_submit(ctx, g, im, not h, o, t)
               for g, im, h, o, t in zip(geoms, imgs, host_mask, outs, tots)]
    try:
        if wait_mode == "poll":
            pending = set(tickets)
            t0 = time.time()
            while pending and time.time() - t0 < 60:
                for tk in list(pending):
                    if dr.dr_poll(ctx, tk) == dr.DR_OK:
                        pending.discard(tk)
                time.sleep(0.001)
            assert not pending, "requests did not complete"
        else:
            for tk in tickets:
                dr.dr_wait(ctx, tk)
        with pytest.raises(dr.DRError) as e:
            dr.dr_poll(ctx, tickets[0])
        assert e.value.code == dr.DR_E_NOTFOUND
        torch.cuda.synchronize()
        return [(o.cpu().numpy(), t.cpu().numpy()) for o, t in zip(outs, tots)]
    finally:
        for g in geoms:
            dr.dr_geometry_free(g)


def test_serving_mix_equals_alone(dr, ctx):
    scans = uneven_scans(9, odd=True)
    singles = [alone(dr, ctx, s) for s in scans]
    served = _serve(dr, ctx, scans, [True, False, True, True, False, True])
    for s, (o1, t1), (o2, t2) in zip(scans, singles, served):
        assert np.array_equal(o2, o1), s.name
        assert_totals_close(t2, t1.astype(np.float64), s.images)
    st = dr.dr_ctx_stats(ctx)
    assert st["completed"] >= len(scans) and st["hbm_in_use"] == 0


def test_serving_tight_budget_queues(dr):
    """A budget that fits about one request at a time: requests wait for
    admission and still produce the same results; an oversized request is
    refused at submission."""
    scans = uneven_scans(10)
    # a request's footprint: its images, its output, its partial totals (at
    # most an eighth of the output here) and their workspace
    biggest = max(s.images.nbytes + 4 * s.grid.n_bins * s.detector.nx * s.detector.ny
                  for s in scans)
    small_ctx = dr.dr_ctx_create(0, int(biggest * 1.5) + (8 << 20))
    try:
        singles = [alone(dr, small_ctx, s) for s in scans]
        served = _serve(dr, small_ctx, scans, [True] * len(scans), wait_mode="wait")
        for s, (o1, t1), (o2, t2) in zip(scans, singles, served):
            assert np.array_equal(o2, o1), s.name
            assert_totals_close(t2, t1.astype(np.float64), s.images)
        import torch
        big = synth.tiny(512, 512, 101, 11, seed=3, n_src=1, noise=False)
        g = dr.dr_geometry_init(small_ctx, big.detector, big.wire, big.grid)
        try:
            out = torch.empty((11, 512, 512), device="cuda")
            with pytest.raises(dr.DRError) as e:
                dr.dr_submit(small_ctx, g, pinned_images(big.images), False, out, None)
            assert e.value.code == dr.DR_E_NOMEM
        finally:
            dr.dr_geometry_free(g)
    finally:
        dr.dr_ctx_destroy(small_ctx)


def mixed_kinds(seed):
    """Scans the persistent kernel takes and scans launched on their own: a
    tilted detector (per-pixel path), step weights, both edges with a tilted
    wire axis."""
    import math
    scans = uneven_scans(seed)[:3]
    s = synth.tiny(150, 5, 31, 81, seed=seed + 1, n_src=8, dark=100.0, render_now=False)
    d = s.detector
    s.detector = synth.Detector(d.nx, d.ny, d.origin, np.array([200.0, 10.0, 30.0]), d.v)
    synth.render(s)
    scans.append(s)
    s = synth.tiny(128, 6, 29, 71, seed=seed + 2, n_src=8, dark=100.0)
    s.wire.weights = np.random.default_rng(seed).uniform(0.5, 2.0, s.wire.n_steps)
    scans.append(s)
    s = synth.tiny(90, 4, 27, 81, seed=seed + 3, n_src=8, dark=100.0, render_now=False)
    t = math.radians(6.0)
    s.wire.axis = np.array([math.cos(t), 0.0, math.sin(t)])
    s.grid = synth.DepthGrid(81, -72.0 + 0.6, 1.2)
    s.wire.edge = synth.EDGE_BOTH
    synth.render(s)
    scans.append(s)
    return scans


def test_batch_and_serving_take_every_kind_of_scan(dr, ctx):
    import torch
    scans = mixed_kinds(21)
    singles = [alone(dr, ctx, s) for s in scans]
    geoms, imgs, outs, tots = [], [], [], []
    for s in scans:
        geoms.append(dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid))
        imgs.append(dev_images(s.images))
        outs.append(torch.full((s.grid.n_bins, s.detector.ny, s.detector.nx), float("nan"),
                               device="cuda"))
        tots.append(torch.full((s.grid.n_bins,), float("nan"), device="cuda"))
    assert [dr.dr_geometry_path(g) for g in geoms][3:] == [dr.DR_PATH_PIXELS, dr.DR_PATH_ROWS,
                                                           dr.DR_PATH_PIXELS]
    torch.cuda.synchronize()
    b = dr.dr_batch_create(ctx, list(zip(geoms, imgs, outs, tots)),
                           dr.DR_BATCH_AUTOTUNE | dr.DR_BATCH_GRAPH)
    try:
        for rep in range(2):
            for o, t in zip(outs, tots):
                o.fill_(float("nan"))
                t.fill_(float("nan"))
            dr.dr_batch_run(b, torch.cuda.current_stream())
            torch.cuda.synchronize()
            for s, (o1, t1), o, t in zip(scans, singles, outs, tots):
                assert np.array_equal(o.cpu().numpy(), o1), (rep, s.name)
                assert_totals_close(t.cpu().numpy(), t1.astype(np.float64), s.images)
    finally:
        dr.dr_batch_free(b)
        for g in geoms:
            dr.dr_geometry_free(g)
    served = _serve(dr, ctx, scans, [True, False, True, True, False, True])
    for s, (o1, t1), (o2, t2) in zip(scans, singles, served):
        assert np.array_equal(o2, o1), s.name
        assert_totals_close(t2, t1.astype(np.float64), s.images)


def test_batch_keeps_its_geometries(dr, ctx):
    """A batch keeps the launch plan it was built with: while it exists its
    geometries can be neither freed nor given step weights."""
    import torch
    s = uneven_scans(31)[0]
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    out = torch.empty((s.grid.n_bins, s.detector.ny, s.detector.nx), device="cuda")
    b = dr.dr_batch_create(ctx, [(g, dev_images(s.images), out, None)], 0)
    try:
        for call in (lambda: dr.dr_geometry_set_step_weights(g, np.ones(s.wire.n_steps)),
                     lambda: dr.dr_geometry_free(g)):
            with pytest.raises(dr.DRError) as e:
                call()
            assert e.value.code == dr.DR_E_BUSY
    finally:
        dr.dr_batch_free(b)
    dr.dr_geometry_set_step_weights(g, np.ones(s.wire.n_steps))
    dr.dr_geometry_free(g)
