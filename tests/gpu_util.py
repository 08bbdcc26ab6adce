"""Helpers for the GPU tests: device buffers through torch, runs through the
C ABI, comparisons against the oracle at the stated tolerance."""
from __future__ import annotations

import numpy as np

# |out_gpu - out_oracle| <= REL_TOL * sum_k |I_k - I_{k+1}| per pixel and bin
REL_TOL = 1e-5


def dev_images(images_u16: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(images_u16).view(np.int16)).to("cuda")


def pinned_images(images_u16: np.ndarray):
    import torch
    t = torch.empty(images_u16.shape, dtype=torch.int16, pin_memory=True)
    t.numpy()[...] = images_u16.view(np.int16)
    return t


def abs_diff_scale(images_u16: np.ndarray) -> np.ndarray:
    """sum_k |I_k - I_{k+1}| per pixel, [ny][nx]."""
    I = images_u16.astype(np.int64)
    return np.abs(np.diff(I, axis=0)).sum(0).astype(np.float64)


def run_f32(dr, ctx, scan, tile=None, totals=True, geom=None, on_device=True, stream=None):
    import torch
    det, grid = scan.detector, scan.grid
    own = geom is None
    g = dr.dr_geometry_init(ctx, det, scan.wire, grid) if own else geom
    try:
        if tile is not None:
            dr.dr_set_tile(g, tile)
        out = torch.full((grid.n_bins, det.ny, det.nx), float("nan"), dtype=torch.float32,
                         device="cuda")
        tot = torch.full((grid.n_bins,), float("nan"), dtype=torch.float32,
                         device="cuda") if totals else None
        img = dev_images(scan.images) if on_device else pinned_images(scan.images)
        dr.dr_reconstruct(g, img, on_device, out, tot,
                          torch.cuda.current_stream() if stream is None else stream)
        torch.cuda.synchronize()
        return out.cpu().numpy(), (tot.cpu().numpy() if totals else None)
    finally:
        if own:
            dr.dr_geometry_free(g)


def run_f64(dr, ctx, scan):
    import torch
    det, grid = scan.detector, scan.grid
    g = dr.dr_geometry_init(ctx, det, scan.wire, grid)
    try:
        out = torch.full((grid.n_bins, det.ny, det.nx), float("nan"), dtype=torch.float64,
                         device="cuda")
        tot = torch.full((grid.n_bins,), float("nan"), dtype=torch.float64, device="cuda")
        img = dev_images(scan.images)
        dr.dr_reconstruct_f64(g, img, out, tot, torch.cuda.current_stream())
        torch.cuda.synchronize()
        return out.cpu().numpy(), tot.cpu().numpy()
    finally:
        dr.dr_geometry_free(g)


def assert_f32_close(out_gpu: np.ndarray, out_ref: np.ndarray, images_u16: np.ndarray):
    scale = abs_diff_scale(images_u16)[None, :, :]
    err = np.abs(out_gpu.astype(np.float64) - out_ref)
    bad = err > REL_TOL * scale
    assert not np.isnan(out_gpu).any(), "unwritten output elements"
    assert not bad.any(), (
        f"{int(bad.sum())} elements off; worst ratio "
        f"{float((err / np.maximum(scale, 1e-300)).max()):.3e}")


def assert_totals_close(tot_gpu: np.ndarray, tot_ref: np.ndarray, images_u16: np.ndarray):
    scale = abs_diff_scale(images_u16).sum()
    err = np.abs(tot_gpu.astype(np.float64) - tot_ref)
    assert not np.isnan(tot_gpu).any()
    assert (err <= REL_TOL * scale).all(), float(err.max() / max(scale, 1e-300))
