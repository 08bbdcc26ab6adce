"""Input generator properties and the paper's row-slab worked example (oracle side)."""
import json
import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_generator_deterministic_and_thread_independent():
    a = synth.tiny(33, 17, 12, 20, seed=5, dark=100.0)
    b = synth.config1()
    s = synth.tiny(33, 17, 12, 20, seed=5, dark=100.0, noise=True)
    again = np.empty_like(s.images)
    synth.render(s, out=again, nthreads=1)
    assert np.array_equal(a.images, again)
    c = synth.config1()
    assert np.array_equal(b.images, c.images)


def test_rows_share_bit_identical_pixel_centres():
    for det in (synth.flat_detector(2048, 2048, 200.0),
                synth.flat_detector(1024, 1024, 400.0),
                synth.flat_detector(256, 256, 200.0, full_nx=2048, full_ny=2048, i0=77, j0=1311)):
        y, z = det.pixel_yz()
        assert np.all(y == y[:, :1]) and np.all(z == z[:, :1])
        assert det.u[1] == 0.0 and det.u[2] == 0.0


def test_wire_scan_geometry():
    w = synth.wire_scan(41, 1.0)
    mid = w.centers[20]
    assert mid[1] == 300.0 and mid[2] == -26.0
    d = np.diff(w.centers, axis=0)
    assert np.allclose(d[:, 1], np.sqrt(0.5)) and np.allclose(d[:, 2], np.sqrt(0.5))


def test_poisson_noise_statistics():
    """Dark-only pixels: counts are Poisson(dark): mean and variance match."""
    s = synth.tiny(64, 64, 40, 10, seed=9, n_src=0, dark=100.0, noise=True, sigma=0.0)
    x = s.images.astype(np.float64).ravel()
    assert abs(x.mean() - 100.0) < 0.3
    assert abs(x.var() - 100.0) < 3.0
    for lam in (3.5, 37.0, 1234.5):  # rates away from the tabulated dark level
        u = synth.tiny(32, 32, 30, 10, seed=10, n_src=0, dark=lam, noise=True, sigma=0.0)
        y = u.images.astype(np.float64).ravel()
        assert abs(y.mean() - lam) < 6 * np.sqrt(lam / y.size) + 0.01 * lam
        assert abs(y.var() / lam - 1.0) < 0.08


def test_worked_example_row_slabs_oracle():
    """4 images x 6 rows x 9 columns reconstructed in three 2-row passes equals
    the single-pass result bit for bit."""
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    n, rows, cols, k = ex["n_images"], ex["n_rows"], ex["n_cols"], ex["rows_per_pass"]
    assert ex["passes"] * k == rows and k * cols * n == ex["threads_per_pass"]
    s = synth.tiny(cols, rows, n, 7, seed=3, pitch=2000.0, step=2.0, width=1.0, n_src=3,
                   dark=20.0)
    full, tot, _ = oracle.reconstruct(s)
    parts = [oracle.reconstruct(s, row0=r, nrows=k)[0] for r in range(0, rows, k)]
    assert np.array_equal(np.concatenate(parts, axis=1), full)
    # thread (row, col, image) = (1, 8, 1) reads element (1, 8, 1) of the slab
    r, c, im = ex["thread_element"]
    slab = s.images[:, 0:k, :]
    flat = slab.reshape(-1)
    assert flat[im * k * cols + r * cols + c] == slab[im, r, c]
