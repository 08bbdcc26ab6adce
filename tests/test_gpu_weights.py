"""Per-step sample weights (monitor normalisation) on the GPU, needs an MI355X.

* FP64 instance bit-exact against the oracle with weights (per-row path,
  generic rows, both edges, per-pixel path, pixel lists);
* FP32 path within 1e-5 of sum_k |I_k w_k - I_{k+1} w_{k+1}| per pixel;
* a stack multiplied by monitor factors in {1, 2} and weighted by their
  reciprocals reconstructs bit for bit like the unmodulated stack;
* host streaming and lists equal the device run; removing the weights
  restores the plain result.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_images, run_f32, run_f64

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


def weighted(s, seed):
    w = np.random.default_rng(seed).uniform(0.5, 2.0, s.wire.n_steps)
    s.wire = synth.Wire(s.wire.radius, s.wire.centers, axis=s.wire.axis, edge=s.wire.edge,
                        weights=w)
    return s


def make_case(name):
    if name == "rows":
        s = synth.tiny(300, 7, 37, 61, seed=501, n_src=12, dark=100.0)
    elif name == "both":
        s = synth.tiny(160, 5, 33, 141, seed=502, n_src=10, dark=100.0)
        s.grid = synth.DepthGrid(141, -71.5 + 0.35, 0.7)
        s.wire.edge = synth.EDGE_BOTH
    elif name == "non_monotone":
        s = synth.tiny(96, 6, 31, 81, seed=503, n_src=8, dark=100.0)
        c = s.wire.centers
        s.wire = synth.Wire(s.wire.radius, np.ascontiguousarray(np.concatenate([c, c[::-1][1:]])))
        synth.render(s)
    elif name == "tilted":
        s = synth.tiny(300, 4, 31, 81, seed=504, n_src=10, dark=100.0, render_now=False)
        d = s.detector
        s.detector = synth.Detector(d.nx, d.ny, d.origin, np.array([200.0, 15.0, 35.0]), d.v)
        synth.render(s)
    else:
        raise KeyError(name)
    return weighted(s, CASES.index(name) + 11)


CASES = ["rows", "both", "non_monotone", "tilted"]


def weighted_scale(s):
    I = s.images.astype(np.float64) * s.wire.weights[:, None, None]
    return np.abs(np.diff(I, axis=0)).sum(0)


@pytest.mark.parametrize("name", CASES)
def test_f64_bit_exact_and_f32_tolerance(dr, ctx, name):
    s = make_case(name)
    ref, tref, _ = oracle.reconstruct(s)
    out64, _ = run_f64(dr, ctx, s)
    assert np.array_equal(out64.view(np.int64), ref.view(np.int64))
    out, tot = run_f32(dr, ctx, s)
    scale = weighted_scale(s)
    assert not np.isnan(out).any()
    assert np.all(np.abs(out.astype(np.float64) - ref) <= 1e-5 * scale[None])
    assert np.all(np.abs(tot.astype(np.float64) - tref) <= 1e-5 * scale.sum())


@pytest.mark.parametrize("name", ["rows", "both", "tilted"])
def test_monitor_modulation_undone_exactly(dr, ctx, name):
    s = make_case(name)
    s.wire.weights = None
    s.images = (s.images // 2).astype(np.uint16)
    plain, _ = run_f32(dr, ctx, s)
    m = np.random.default_rng(7).integers(1, 3, s.wire.n_steps)
    mod = synth.Scan(s.name, s.detector, synth.Wire(s.wire.radius, s.wire.centers,
                                                    axis=s.wire.axis, edge=s.wire.edge,
                                                    weights=1.0 / m),
                     s.grid, s.sources, s.dark, s.noise, s.seed,
                     images=(s.images.astype(np.int64) * m[:, None, None]).astype(np.uint16))
    got, _ = run_f32(dr, ctx, mod)
    assert np.array_equal(got, plain)


@pytest.mark.parametrize("name", ["rows", "tilted"])
def test_streaming_lists_and_removal(dr, ctx, name, monkeypatch):
    import torch
    s = make_case(name)
    g = dr.dr_geometry_init(ctx, s.detector, s.wire, s.grid)
    try:
        dev, _ = run_f32(dr, ctx, s, geom=g)
        monkeypatch.setenv("DR_SLAB_ROWS", "2")
        host, _ = run_f32(dr, ctx, s, geom=g, on_device=False)
        assert np.array_equal(host, dev)
        pix = np.arange(0, s.detector.nx * s.detector.ny, 3)
        lst = dr.dr_list_create(g, pix)
        try:
            out = torch.empty((s.grid.n_bins, pix.shape[0]), device="cuda")
            dr.dr_reconstruct_list(lst, dev_images(s.images), dr.DR_LAYOUT_FULL, True, out, None,
                                   torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), dev.reshape(s.grid.n_bins, -1)[:, pix])
            out64 = torch.empty((s.grid.n_bins, pix.shape[0]), dtype=torch.float64,
                                device="cuda")
            dr.dr_reconstruct_list_f64(lst, dev_images(s.images), dr.DR_LAYOUT_FULL, out64, None,
                                       torch.cuda.current_stream())
            torch.cuda.synchronize()
            ref, _, _ = oracle.reconstruct_pixels(s, pix, want_bins=False)
            assert np.array_equal(out64.cpu().numpy().T.view(np.int64), ref.view(np.int64))
        finally:
            dr.dr_list_free(lst)
        with pytest.raises(dr.DRError) as e:
            dr.dr_geometry_set_step_weights(g, np.full(s.wire.n_steps, np.nan))
        assert e.value.code == dr.DR_E_INVAL
        dr.dr_geometry_set_step_weights(g, None)
        unweighted, _ = run_f32(dr, ctx, s, geom=g)
        s.wire.weights = None
        fresh, _ = run_f32(dr, ctx, s)
        assert np.array_equal(unweighted, fresh)
    finally:
        dr.dr_geometry_free(g)
