"""Parity at the sizes the benchmark times (needs an MI355X).

* the 16-scan batched workload (seed 4: ROI sides 256-1024 px, 101-801 steps,
  201-801 bins) in one autotuned, graph-captured persistent launch: every
  scan's output bitwise equal to its single-scan call, and >= 2000 sampled
  pixels per scan within 1e-5 * sum_k |dI_k| of the oracle;
* the full-frame scan (2048^2 px, 1001 steps, 1001 bins) from pinned host
  memory (row slabs double-buffered over PCIe) bitwise equal to the run from
  images resident in HBM;
* a serving mix holding that full-frame host-image request between small
  requests: each output bitwise equal to its run alone, and sampled pixels of
  the full frame against the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, dev_images, pinned_images

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


def sample(nx, ny, n, seed):
    rng = np.random.default_rng(seed)
    edge = [0, nx - 1, (ny - 1) * nx, ny * nx - 1]
    return np.unique(np.concatenate([edge, rng.integers(0, nx * ny, n)]))


def check_sampled(scan, out_dev, pix):
    """Sampled pixels of a device output [B][ny][nx] against the oracle."""
    import torch
    N, B = scan.wire.n_steps, scan.grid.n_bins
    ref, _, _ = oracle.reconstruct_pixels(scan, pix, want_bins=False)
    got = out_dev.view(B, -1)[:, torch.from_numpy(pix).to(out_dev.device)].T.cpu().numpy()
    series = scan.images.reshape(N, -1)[:, pix].T.astype(np.int64)
    scale = np.abs(np.diff(series, axis=1)).sum(1).astype(np.float64)
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= REL_TOL * scale[:, None]), (
        scan.name, float((err / np.maximum(scale[:, None], 1e-300)).max()))


def total_scale(images, rows=64):
    """sum over pixels and steps of |I_k - I_{k+1}|, computed on the device in
    row blocks from a [N][ny][nx] int16 tensor (host or device) of uint16
    counts."""
    import torch
    total = 0.0
    for r0 in range(0, images.shape[1], rows):
        blk = images[:, r0:r0 + rows].to("cuda").to(torch.int32) & 0xFFFF
        total += float((blk[1:] - blk[:-1]).abs().sum(dtype=torch.float64))
    return total


def device_equal(a, b, rows=64):
    """Bitwise equality of two device tensors [B][ny][nx], in row blocks."""
    import torch
    for r0 in range(0, a.shape[1], rows):
        if not torch.equal(a[:, r0:r0 + rows].view(torch.int32), b[:, r0:r0 + rows].view(torch.int32)):
            return False
    return True


def test_batched_workload_full_size(dr, ctx):
    import torch
    scans = synth.config4()
    stream = torch.cuda.current_stream()
    geoms, imgs, outs, tots = [], [], [], []
    try:
        for s in scans:
            geoms.append(dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid))
            imgs.append(dev_images(s.images))
            outs.append(torch.full((s.grid.n_bins, s.detector.ny, s.detector.nx), float("nan"),
                                   device="cuda"))
            tots.append(torch.full((s.grid.n_bins,), float("nan"), device="cuda"))
        torch.cuda.synchronize()
        b = dr.dr_batch_create(ctx, list(zip(geoms, imgs, outs, tots)),
                               dr.DR_BATCH_AUTOTUNE | dr.DR_BATCH_GRAPH)
        try:
            for o, t in zip(outs, tots):
                o.fill_(float("nan"))
                t.fill_(float("nan"))
            dr.dr_batch_run(b, stream)
            torch.cuda.synchronize()
        finally:
            dr.dr_batch_free(b)
        for n, (s, g, img, o, t) in enumerate(zip(scans, geoms, imgs, outs, tots)):
            single = torch.full_like(o, float("nan"))
            tsingle = torch.full_like(t, float("nan"))
            dr.dr_reconstruct(g, img, True, single, tsingle, stream)
            torch.cuda.synchronize()
            assert device_equal(o, single), s.name
            scale = total_scale(img)
            assert float((t.double() - tsingle.double()).abs().max()) <= REL_TOL * scale, s.name
            del single
            check_sampled(s, o, sample(s.detector.nx, s.detector.ny, 2000, 40 + n))
    finally:
        for g in geoms:
            dr.dr_geometry_free(g)
        del imgs, outs
        torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def full_frame():
    import torch
    s = synth.config3(render_now=False)
    host = torch.empty((s.wire.n_steps, s.detector.ny, s.detector.nx), dtype=torch.int16,
                       pin_memory=True)
    synth.render(s, out=host.numpy().view(np.uint16))
    s.images = host.numpy().view(np.uint16)
    return s, host


def test_full_frame_from_host_equals_resident(dr, ctx, full_frame):
    import torch
    s, host = full_frame
    B, ny, nx = s.grid.n_bins, s.detector.ny, s.detector.nx
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    stream = torch.cuda.current_stream()
    try:
        dev = host.to("cuda")
        ref = torch.full((B, ny, nx), float("nan"), device="cuda")
        tref = torch.full((B,), float("nan"), device="cuda")
        dr.dr_reconstruct(g, dev, True, ref, tref, stream)
        del dev
        out = torch.full((B, ny, nx), float("nan"), device="cuda")
        tot = torch.full((B,), float("nan"), device="cuda")
        dr.dr_reconstruct(g, host, False, out, tot, stream)
        torch.cuda.synchronize()
        assert device_equal(out, ref)
        assert torch.equal(tot, tref)
        check_sampled(s, out, sample(nx, ny, 2000, 51))
    finally:
        dr.dr_geometry_free(g)
        torch.cuda.empty_cache()


def test_serving_mix_with_full_frame(dr, ctx, full_frame):
    import time
    import torch
    s_full, host_full = full_frame
    small = []
    rng = np.random.default_rng(np.random.SeedSequence(52))
    for n in range(6):
        side = int(rng.choice([128, 256]))
        N, B = int(rng.integers(101, 302)), int(rng.integers(201, 402))
        i0, j0 = (int(x) for x in rng.integers(0, 2048 - side, 2))
        det = synth.flat_detector(side, side, 200.0, full_nx=2048, full_ny=2048, i0=i0, j0=j0)
        half = 0.5 * min((N - 1) * 0.5 * 0.7, (B - 2) * 0.5)
        src = synth.draw_sources(rng, max(2, side * side // 500), side, side, -half, half)
        s = synth.Scan(f"small{n}", det, synth.wire_scan(N, 0.5), synth.centered_grid(B, 0.5),
                       src, dark=100.0, noise=True, seed=5200 + n)
        synth.render(s)
        small.append(s)
    scans = small[:3] + [s_full] + small[3:]
    host_mask = [True, False, True, True, True, False, True]
    stream = torch.cuda.current_stream()
    geoms = [dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid) for s in scans]
    alone, outs = [], []
    try:
        imgs = []
        for s, h in zip(scans, host_mask):
            if s is s_full:
                imgs.append(host_full)
            else:
                imgs.append(pinned_images(s.images) if h else dev_images(s.images))
        # each request alone: the single-scan call, host images streamed
        alone = []
        for g, s, im, h in zip(geoms, scans, imgs, host_mask):
            o = torch.full((s.grid.n_bins, s.detector.ny, s.detector.nx), float("nan"),
                           device="cuda")
            t = torch.full((s.grid.n_bins,), float("nan"), device="cuda")
            dr.dr_reconstruct(g, im, not h, o, t, stream)
            alone.append((o, t))
        torch.cuda.synchronize()
        outs = [torch.full_like(o, float("nan")) for o, _ in alone]
        tots = [torch.full_like(t, float("nan")) for _, t in alone]
        # the requests' work is not ordered after torch's stream: the fills
        # above must be complete before submission
        torch.cuda.synchronize()
        tickets = [dr.dr_submit(ctx, g, im, not h, o, t)
                   for g, im, h, o, t in zip(geoms, imgs, host_mask, outs, tots)]
        pending, t0 = set(tickets), time.time()
        while pending and time.time() - t0 < 90:
            for tk in list(pending):
                if dr.dr_poll(ctx, tk) == dr.DR_OK:
                    pending.discard(tk)
            time.sleep(0.001)
        assert not pending, "requests did not complete"
        torch.cuda.synchronize()
        for s, im, (o1, t1), o2, t2 in zip(scans, imgs, alone, outs, tots):
            assert device_equal(o2, o1), s.name
            scale = total_scale(im)
            assert float((t2.double() - t1.double()).abs().max()) <= REL_TOL * scale, s.name
        check_sampled(s_full, outs[3], sample(2048, 2048, 2000, 53))
        check_sampled(small[0], outs[0], sample(small[0].detector.nx, small[0].detector.ny, 500, 54))
    finally:
        del alone, outs
        for g in geoms:
            dr.dr_geometry_free(g)
        torch.cuda.empty_cache()
