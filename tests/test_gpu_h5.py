"""Files to depth images on the GPU (needs an MI355X and the HDF5 layer):
a scan written as one HDF5 file per wire step, read back into pinned memory
(whole or in row slabs), reconstructed from host memory, must equal the
reconstruction of the in-memory stack bit for bit; the depth images written
back read the same."""
import os

import numpy as np
import pytest

import synth
from gpu_util import run_f32
from paper_2201_13309_amd import build as pkg_build

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not pkg_build.hdf5_available(), reason="no HDF5 installation")]


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


@pytest.mark.parametrize("deflate", [0, 3])
def test_files_to_depth_images(dr, ctx, tmp_path, monkeypatch, deflate):
    import torch
    from paper_2201_13309_amd import dr_h5
    s = synth.tiny(200, 13, 41, 101, seed=401, n_src=12, dark=100.0)
    N, ny, nx = s.images.shape
    paths = [str(tmp_path / f"scan_{k:04d}.h5") for k in range(N)]
    dr_h5.write_stack(paths, "/entry1/data/data", s.images, deflate=deflate)
    dr_h5.write_scalars(paths, "/entry1/wire/y", s.wire.centers[:, 1])
    dr_h5.write_scalars(paths, "/entry1/wire/z", s.wire.centers[:, 2])
    st = dr_h5.open_stack(paths, "/entry1/data/data")
    try:
        host = torch.empty((N, ny, nx), dtype=torch.int16, pin_memory=True)
        for r0 in range(0, ny, 5):  # row slabs of every file
            nr = min(5, ny - r0)
            slab = np.empty((N, nr, nx), np.uint16)
            dr_h5.read_rows(st, r0, nr, slab)
            host.numpy()[:, r0:r0 + nr] = slab.view(np.int16)
    finally:
        dr_h5.close_stack(st)
    centers = s.wire.centers.copy()
    centers[:, 1] = dr_h5.read_scalars(paths, "/entry1/wire/y")
    centers[:, 2] = dr_h5.read_scalars(paths, "/entry1/wire/z")
    assert np.array_equal(centers, s.wire.centers)
    ref, tref = run_f32(dr, ctx, s)
    g = dr.dr_geometry_init(ctx, s.detector, synth.Wire(s.wire.radius, centers), s.grid)
    try:
        monkeypatch.setenv("DR_SLAB_ROWS", "4")
        out = torch.full((s.grid.n_bins, ny, nx), float("nan"), device="cuda")
        tot = torch.full((s.grid.n_bins,), float("nan"), device="cuda")
        dr.dr_reconstruct(g, host, False, out, tot, torch.cuda.current_stream())
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert np.array_equal(o, ref)
        assert np.array_equal(tot.cpu().numpy(), tref)
    finally:
        dr.dr_geometry_free(g)
    p = str(tmp_path / "depth.h5")
    dr_h5.write_depth_images(p, "/depth_images", o, s.grid.first_center, s.grid.width)
    import subprocess
    dump = str(tmp_path / "depth.bin")
    subprocess.run([os.path.join(pkg_build.HDF5_ROOT, "bin", "h5dump"), "-d", "/depth_images",
                    "-b", "LE", "-o", dump, p], check=True, capture_output=True)
    assert np.array_equal(np.fromfile(dump, dtype="<f4"), o.ravel())
