"""HDF5 file layer (libdr_h5.so), no GPU needed.

Independent checks: files written by the HDF5 command-line importer are read
back by the layer, and files the layer writes are dumped by the HDF5
command-line dumper; both compared byte for byte with the source arrays.
The direct (positioned-read) and library paths agree; the paper's worked
example (4 images x 6 rows x 9 columns, Sec. III-B) read in 2-row slabs
reassembles the stack.
"""
import os
import subprocess

import numpy as np
import pytest

from paper_2201_13309_amd import build as pkg_build

pytestmark = pytest.mark.skipif(not pkg_build.hdf5_available(), reason="no HDF5 installation")

H5BIN = os.path.join(pkg_build.HDF5_ROOT, "bin")


@pytest.fixture(scope="module")
def h5():
    from paper_2201_13309_amd import dr_h5
    if not os.path.exists(dr_h5.LIB_PATH):
        pkg_build.build_h5()
    dr_h5.load()
    return dr_h5


def h5import(tmp, path, dataset, arr, klass="UIN"):
    """Write arr with the HDF5 importer tool (independent of the layer)."""
    raw = os.path.join(tmp, os.path.basename(path) + ".bin")
    np.ascontiguousarray(arr).astype(arr.dtype.newbyteorder("<")).tofile(raw)
    cfg = os.path.join(tmp, os.path.basename(path) + ".cfg")
    size = arr.dtype.itemsize * 8
    open(cfg, "w").write(
        f"PATH {dataset}\nINPUT-CLASS {klass}\nINPUT-SIZE {size}\nINPUT-BYTE-ORDER LE\n"
        f"RANK {arr.ndim}\nDIMENSION-SIZES {' '.join(str(d) for d in arr.shape)}\n"
        f"OUTPUT-CLASS {klass}\nOUTPUT-SIZE {size}\nOUTPUT-ARCHITECTURE STD\n"
        f"OUTPUT-BYTE-ORDER LE\n")
    subprocess.run([os.path.join(H5BIN, "h5import"), raw, "-c", cfg, "-o", path], check=True,
                   capture_output=True)


def h5dump(tmp, path, dataset, dtype):
    """Raw little-endian values of a dataset, by the HDF5 dumper tool."""
    out = os.path.join(tmp, "dump.bin")
    subprocess.run([os.path.join(H5BIN, "h5dump"), "-d", dataset, "-b", "LE", "-o", out, path],
                   check=True, capture_output=True)
    return np.fromfile(out, dtype=np.dtype(dtype).newbyteorder("<"))


def stack(seed, n, ny, nx):
    return np.random.default_rng(seed).integers(0, 65536, (n, ny, nx)).astype(np.uint16)


def test_reads_importer_files(h5, tmp_path):
    imgs = stack(1, 5, 7, 13)
    paths = [str(tmp_path / f"img_{k}.h5") for k in range(5)]
    for p, im in zip(paths, imgs):
        h5import(str(tmp_path), p, "/entry1/data/data", im)
    s = h5.open_stack(paths, "/entry1/data/data")
    try:
        assert h5.stack_shape(s)[:3] == (5, 7, 13)
        out = np.zeros((5, 7, 13), np.uint16)
        h5.read_rows(s, 0, 7, out)
        assert np.array_equal(out, imgs)
        part = np.zeros((5, 3, 13), np.uint16)
        h5.read_rows(s, 4, 3, part, nthreads=2)
        assert np.array_equal(part, imgs[:, 4:7])
    finally:
        h5.close_stack(s)


def test_rank3_single_image_dataset(h5, tmp_path):
    imgs = stack(2, 3, 4, 6)
    paths = [str(tmp_path / f"r3_{k}.h5") for k in range(3)]
    for p, im in zip(paths, imgs):
        h5import(str(tmp_path), p, "/data", im[None])
    s = h5.open_stack(paths, "/data")
    try:
        out = np.zeros((3, 4, 6), np.uint16)
        h5.read_rows(s, 0, 4, out)
        assert np.array_equal(out, imgs)
    finally:
        h5.close_stack(s)


def test_writer_checked_by_dumper(h5, tmp_path):
    imgs = stack(3, 4, 9, 11)
    for deflate in (0, 6):
        paths = [str(tmp_path / f"w{deflate}_{k}.h5") for k in range(4)]
        h5.write_stack(paths, "/entry1/data/data", imgs, deflate=deflate)
        for p, im in zip(paths, imgs):
            assert np.array_equal(h5dump(str(tmp_path), p, "/entry1/data/data", np.uint16),
                                  im.ravel())


def test_direct_and_library_paths_agree(h5, tmp_path):
    imgs = stack(4, 6, 70, 33)  # 70 rows: two deflate chunks of 64 rows
    paths = [str(tmp_path / f"m_{k}.h5") for k in range(6)]
    h5.write_stack(paths[:3], "/d", imgs[:3], deflate=0)
    h5.write_stack(paths[3:], "/d", imgs[3:], deflate=4)
    s = h5.open_stack(paths, "/d")
    try:
        assert h5.stack_shape(s) == (6, 70, 33, 3)
        for row0, nrows in ((0, 70), (0, 1), (63, 2), (69, 1), (10, 55)):
            out = np.zeros((6, nrows, 33), np.uint16)
            h5.read_rows(s, row0, nrows, out, nthreads=4)
            assert np.array_equal(out, imgs[:, row0:row0 + nrows]), (row0, nrows)
    finally:
        h5.close_stack(s)


def test_paper_worked_example_slabs(h5, tmp_path):
    """4 images of 6 rows x 9 columns read 2 rows at a time (Sec. III-B)."""
    imgs = stack(5, 4, 6, 9)
    paths = [str(tmp_path / f"ex_{k}.h5") for k in range(4)]
    h5.write_stack(paths, "/data", imgs)
    s = h5.open_stack(paths, "/data")
    try:
        slabs = []
        for r0 in range(0, 6, 2):
            out = np.zeros((4, 2, 9), np.uint16)
            h5.read_rows(s, r0, 2, out)
            slabs.append(out)
        assert np.array_equal(np.concatenate(slabs, axis=1), imgs)
    finally:
        h5.close_stack(s)


def test_scalars(h5, tmp_path):
    imgs = stack(6, 3, 2, 2)
    paths = [str(tmp_path / f"sc_{k}.h5") for k in range(3)]
    h5.write_stack(paths, "/data", imgs)
    vals = np.array([-12.5, 0.0, 3.25e3])
    h5.write_scalars(paths, "/entry1/wire/y", vals)
    assert np.array_equal(h5.read_scalars(paths, "/entry1/wire/y"), vals)
    for k, p in enumerate(paths):  # an integer array of one element, by the importer
        h5import(str(tmp_path), str(tmp_path / f"mon_{k}.h5"), "/monitor",
                 np.array([1000 + k], dtype=np.int32), klass="IN")
    mon = [str(tmp_path / f"mon_{k}.h5") for k in range(3)]
    assert np.array_equal(h5.read_scalars(mon, "/monitor"), [1000.0, 1001.0, 1002.0])


def test_depth_images_checked_by_dumper(h5, tmp_path):
    out = np.random.default_rng(7).standard_normal((5, 3, 4)).astype(np.float32)
    p = str(tmp_path / "depth.h5")
    h5.write_depth_images(p, "/result/depth_images", out, first_center=-2.0, width=0.5)
    assert np.array_equal(h5dump(str(tmp_path), p, "/result/depth_images", np.float32),
                          out.ravel())
    assert np.array_equal(h5dump(str(tmp_path), p, "/result/depth_images_depth", np.float64),
                          -2.0 + 0.5 * np.arange(5))


def test_large_depth_images(h5, tmp_path):
    """A 30 MB result: every value where the library's own dumper reads it,
    and the depth axis beside it."""
    out = np.random.default_rng(8).standard_normal((3, 1500, 1700)).astype(np.float32)
    p = str(tmp_path / "big.h5")
    h5.write_depth_images(p, "/r/d", out, first_center=1.0, width=0.25)
    assert np.array_equal(h5dump(str(tmp_path), p, "/r/d", np.float32), out.ravel())
    assert np.array_equal(h5dump(str(tmp_path), p, "/r/d_depth", np.float64),
                          1.0 + 0.25 * np.arange(3))
    # rewriting a smaller result into the same path truncates the file first
    small = out[:1, :10, :20].copy()
    h5.write_depth_images(p, "/r/d", small, first_center=0.0, width=1.0)
    assert np.array_equal(h5dump(str(tmp_path), p, "/r/d", np.float32), small.ravel())


def test_errors(h5, tmp_path):
    from paper_2201_13309_amd.dr import DRError, DR_E_INVAL
    a = [str(tmp_path / f"e_{k}.h5") for k in range(2)]
    h5.write_stack(a[:1], "/d", stack(8, 1, 4, 5))
    h5.write_stack(a[1:], "/d", stack(8, 1, 4, 6))  # other width
    for paths, ds in ((a, "/d"), (a[:1], "/missing"), ([str(tmp_path / "none.h5")], "/d")):
        with pytest.raises(DRError) as e:
            h5.open_stack(paths, ds)
        assert e.value.code == DR_E_INVAL
    i32 = str(tmp_path / "i32.h5")
    h5import(str(tmp_path), i32, "/d", np.zeros((4, 5), np.int32), klass="IN")
    with pytest.raises(DRError):
        h5.open_stack([i32], "/d")
    s = h5.open_stack(a[:1], "/d")
    try:
        with pytest.raises(DRError):
            h5.read_rows(s, 3, 2, np.zeros((1, 2, 5), np.uint16))
    finally:
        h5.close_stack(s)


def test_exports(h5):
    lib = h5.load()
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "include", "dr_h5.h")).read()
    import re
    declared = set(re.findall(r"^\s*(?:dr_status|const char\*)\s+(dr_h5_\w+)\s*\(", text, re.M))
    assert declared == set(h5.ABI_SYMBOLS)
    assert all(hasattr(lib, n) for n in declared)
