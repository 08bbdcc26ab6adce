"""Pins of the FP64 oracle to facts other than itself.

Each function takes an oracle library handle (so the mutation test can run the
same checks against a copy of the oracle with a planted mistake) and raises
AssertionError when the pin does not hold.

Independent facts used:
* similar triangles when the pixel is level with the wire centre;
* the zero-radius limit: the ray through the wire centre, a textbook
  line-line intersection;
* bisection on an occlusion predicate (distance from the wire centre to the
  source-pixel segment), written here and never using the tangent formula;
* mirror symmetry about the horizontal line through the wire centre;
* hand-computed bin profiles;
* intensity conservation (sum over bins equals first minus last count);
* brute-force sub-sampled ray integration;
* depths planted by the forward model.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import synth

# ------------------------------------------------------------------ helpers


def seg_dist(cy, cz, zs, py, pz):
    """Distance (y, z projection) from (cy, cz) to the segment (0, zs)-(py, pz)."""
    dy, dz = py, pz - zs
    wy, wz = cy, cz - zs
    t = (wy * dy + wz * dz) / (dy * dy + dz * dz)
    t = min(1.0, max(0.0, t))
    return math.hypot(wy - t * dy, wz - t * dz)


def seg_dist_vec(cy, cz, zs: np.ndarray, py, pz) -> np.ndarray:
    dy = py
    dz = pz - zs
    wy = cy
    wz = cz - zs
    t = np.clip((wy * dy + wz * dz) / (dy * dy + dz * dz), 0.0, 1.0)
    return np.hypot(wy - t * dy, wz - t * dz)


def random_geometries(n, seed):
    """Random pixel/wire placements spanning the workloads' ranges (um)."""
    rng = np.random.default_rng(seed)
    py = rng.uniform(2.0e5, 8.0e5, n)
    pz = rng.uniform(-3.0e5, 3.0e5, n)
    cy = rng.uniform(50.0, 2000.0, n)
    cz = rng.uniform(-500.0, 500.0, n)
    r = rng.uniform(5.0, 100.0, n)
    return py, pz, cy, cz, r


# -------------------------------------------------------- tangent depth pins


def pin_closed_form_level(lib):
    """Pixel level with the wire centre (Pz = Cz): similar triangles give
    d = Cz + s r Py / sqrt((Py - Cy)^2 - r^2)."""
    py, _, cy, cz, r = random_geometries(500, 11)
    for s in (+1, -1):
        for a, b, c, rr in zip(py, cy, cz, r):
            d = oracle.tangent_depth(a, c, b, c, rr, s, lib=lib)
            ref = c + s * rr * a / math.sqrt((a - b) ** 2 - rr * rr)
            assert abs(d - ref) <= 1e-9 * (1.0 + abs(ref)), (d, ref)
    # numbers of the 510 mm geometry: +-26.0153 um about the wire centre
    d = oracle.tangent_depth(510000.0, -26.0, 300.0, -26.0, 26.0, +1, lib=lib)
    assert abs((d + 26.0) - 26.0153) < 1e-4, d


def pin_zero_radius(lib):
    """r -> 0: the ray through the wire centre, d = Cz - Cy (Cz - Pz)/(Cy - Py)."""
    py, pz, cy, cz, _ = random_geometries(500, 12)
    for s in (+1, -1):
        for a, z, b, c in zip(py, pz, cy, cz):
            d = oracle.tangent_depth(a, z, b, c, 1e-300, s, lib=lib)
            ref = c - b * (c - z) / (b - a)
            assert abs(d - ref) <= 1e-9 * (1.0 + abs(ref)), (d, ref)


def pin_bisection(lib):
    """Tangent depth equals the beam point where the source-pixel segment just
    touches the wire disc, found by bisection on the distance alone."""
    py, pz, cy, cz, r = random_geometries(300, 13)
    for a, z, b, c, rr in zip(py, pz, cy, cz, r):
        zc = c - b * (c - z) / (b - a)  # segment through the wire centre
        for s in (+1, -1):
            # on side s the distance grows from 0 (at zc) past r; bracket it
            lo, hi = zc, zc + s * 1e4
            assert seg_dist(b, c, hi, a, z) > rr
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if seg_dist(b, c, mid, a, z) < rr:
                    lo = mid
                else:
                    hi = mid
            d = oracle.tangent_depth(a, z, b, c, rr, s, lib=lib)
            assert abs(d - 0.5 * (lo + hi)) < 2e-8, (d, lo, hi, s)


def pin_mirror(lib):
    """Reflecting z about the wire centre swaps the two edges:
    d_s(Pz) = 2 Cz - d_{-s}(2 Cz - Pz)."""
    py, pz, cy, cz, r = random_geometries(500, 14)
    for a, z, b, c, rr in zip(py, pz, cy, cz, r):
        for s in (+1, -1):
            d1 = oracle.tangent_depth(a, z, b, c, rr, s, lib=lib)
            d2 = oracle.tangent_depth(a, 2 * c - z, b, c, rr, -s, lib=lib)
            assert abs(d1 - (2 * c - d2)) <= 1e-9 * (1.0 + abs(d1)), (d1, d2)


def pin_edge_sign(lib):
    """The leading edge is the +z edge when the wire moves downstream (+z) and
    the -z edge when the same scan runs backwards."""
    w = synth.wire_scan(41, 1.0)
    assert oracle.edge_sign(510000.0, 0.0, w.centers, 26.0, lib=lib) == +1
    assert oracle.edge_sign(510000.0, 0.0, w.centers[::-1].copy(), 26.0, lib=lib) == -1


# ---------------------------------------------------------------- binning pins

HAND_PROFILES = [
    # (u, I, n_bins, expected out) -- computed by hand
    ([0.5, 1.5], [10, 0], 3, [5.0, 5.0, 0.0]),            # split evenly over two bins
    ([1.25, 1.75], [8, 2], 3, [0.0, 6.0, 0.0]),           # inside one bin: fraction 1
    ([-0.5, 0.5], [10, 0], 3, [5.0, 0.0, 0.0]),           # part below the grid dropped
    ([2.5, 3.5], [10, 0], 3, [0.0, 0.0, 5.0]),            # part above the grid dropped
    ([1.0, 2.0], [4, 0], 4, [0.0, 4.0, 0.0, 0.0]),        # exact bin edges: one bin
    ([1.3, 1.3], [4, 1], 3, [0.0, 3.0, 0.0]),             # zero length: point mass
    ([2.5, 0.5], [10, 0], 3, [2.5, 5.0, 2.5]),            # decreasing positions
    ([0.0, 4.0], [0, 8], 4, [-2.0, -2.0, -2.0, -2.0]),    # negative difference kept
    ([0.5, 1.5, 3.0], [10, 4, 1], 4, [3.0, 3.0 + 1.0, 2.0, 0.0]),
    ([-5.0, -4.0], [9, 0], 3, [0.0, 0.0, 0.0]),           # entirely outside
    ([3.0, 5.0], [9, 0], 3, [0.0, 0.0, 0.0]),             # starts at the top edge
    ([0.0, 0.0], [6, 1], 2, [5.0, 0.0]),                  # zero length at bin edge 0
    ([-1.0, 0.0], [6, 1], 2, [0.0, 0.0]),                 # ends exactly at the grid start
]


def pin_hand_profiles(lib):
    for u, I, B, want in HAND_PROFILES:
        got = oracle.bin_profile(u, I, B, lib=lib)
        assert np.allclose(got, want, rtol=0, atol=1e-12), (u, I, got, want)


def pin_conservation_random(lib):
    """Positions inside the grid: the profile sums to I_0 - I_{N-1}."""
    rng = np.random.default_rng(15)
    for _ in range(50):
        N = int(rng.integers(2, 60))
        B = 50
        u = np.sort(rng.uniform(0.0, B, N))
        if rng.random() < 0.5:
            u = u[::-1].copy()
        I = rng.integers(0, 65536, N).astype(np.float64)
        got = oracle.bin_profile(u, I, B, lib=lib)
        assert abs(got.sum() - (I[0] - I[-1])) <= 1e-8 * (1 + np.abs(np.diff(I)).sum())


# --------------------------------------------------------- whole-chain pins


def pin_conservation_scan(lib):
    """Config-1 scan: every pixel's sweep lies inside the grid, so each pixel
    conserves intensity (leading: I_0 - I_{N-1}; trailing: I_{N-1} - I_0;
    their average: 0) and the totals sum to the total of the same."""
    s = synth.config1()
    s.grid = synth.centered_grid(201, 1.0)  # wide enough for the trailing sweep too
    I = s.images.astype(np.float64)
    scale = np.abs(np.diff(I, axis=0)).sum(0) + 1.0
    for edge, want in ((synth.EDGE_LEADING, I[0] - I[-1]), (synth.EDGE_TRAILING, I[-1] - I[0]),
                       (synth.EDGE_BOTH, 0.0 * I[0])):
        s.wire.edge = edge
        out, tot, bins = oracle.reconstruct(s, want_bins=True, lib=lib)
        assert bins.min() >= 0 and bins.max() <= s.grid.n_bins - 1
        assert np.all(np.abs(out.sum(0) - want) <= 1e-9 * scale), edge
        assert abs(tot.sum() - want.sum()) <= 1e-9 * scale.sum(), edge


def brute_force_pixel(py, pz, centers, r, grid, I, samples_per_bin=4000, edge=0):
    """Depth profile of one pixel by sub-sampling the beam.  Leading edge: the
    intensity lost between steps k and k+1 is spread uniformly over the beam
    points that are clear at step k and blocked at step k+1 (the slice the
    leading edge covers).  Trailing edge: the intensity regained is spread over
    the points blocked at k and clear at k+1.  Both: the average of the two.
    Returns (profile, per-bin error bound)."""
    if edge == synth.EDGE_BOTH:
        p1, e1 = brute_force_pixel(py, pz, centers, r, grid, I, samples_per_bin, 0)
        p2, e2 = brute_force_pixel(py, pz, centers, r, grid, I, samples_per_bin, 1)
        return 0.5 * (p1 + p2), 0.5 * (e1 + e2)
    B, w, c0 = grid.n_bins, grid.width, grid.first_center
    e0 = c0 - 0.5 * w
    h = w / samples_per_bin
    # sample far beyond the grid so that slices crossing its ends are measured whole
    zlo, zhi = e0 - 30.0 * w, e0 + (B + 30) * w
    z = zlo + h * (np.arange(int((zhi - zlo) / h)) + 0.5)
    occ = np.stack([seg_dist_vec(c[1], c[2], z, py, pz) < r for c in centers])
    binidx = np.floor((z - e0) / w).astype(np.int64)
    inside = (binidx >= 0) & (binidx < B)
    prof = np.zeros(B)
    err = np.zeros(B)
    for k in range(len(centers) - 1):
        if edge == synth.EDGE_TRAILING:
            newly = occ[k] & ~occ[k + 1]
            dI = float(I[k + 1]) - float(I[k])
        else:
            newly = occ[k + 1] & ~occ[k]
            dI = float(I[k]) - float(I[k + 1])
        n = int(newly.sum())
        if n == 0:
            continue
        sel = newly & inside
        cnt = np.bincount(binidx[sel], minlength=B)
        prof += dI * cnt / n
        touched = cnt > 0
        err[touched] += abs(dI) * 4.0 / n
    return prof, err


def pin_brute_force(lib):
    """Tiny scans (4x4 px, 9 steps, 15 bins) against brute-force integration,
    for the leading edge, the trailing edge and their average: every pixel's
    profile, and the per-depth totals bin by bin against the sum of the
    brute-force profiles over the pixels (within the summed bounds)."""
    shaped = 0
    for seed, step, width, edge in ((21, 1.0, 1.0, 0), (22, 0.5, 0.5, 0), (23, 2.0, 1.0, 0),
                                    (24, 1.0, 1.0, 1), (25, 2.0, 1.0, 2)):
        s = synth.tiny(4, 4, 9, 15, seed=seed, pitch=3000.0, step=step, width=width,
                       n_src=6, dark=50.0, sigma=1.0)
        s.wire.edge = edge
        out, tot, _ = oracle.reconstruct(s, lib=lib)
        py, pz = s.detector.pixel_yz()
        tot_bf = np.zeros(s.grid.n_bins)
        tot_err = np.zeros(s.grid.n_bins)
        for j in range(4):
            for i in range(4):
                prof, err = brute_force_pixel(py[j, i], pz[j, i], s.wire.centers,
                                              s.wire.radius, s.grid, s.images[:, j, i],
                                              edge=edge)
                got = out[:, j, i]
                assert np.all(np.abs(got - prof) <= err + 1e-9), (seed, j, i, got, prof, err)
                tot_bf += prof
                tot_err += err
        assert np.all(np.abs(tot - tot_bf) <= tot_err + 1e-8), (seed, tot, tot_bf, tot_err)
        # totals far from flat, so that a shifted or permuted bin index fails
        shaped += np.abs(np.diff(tot_bf)).max() > 100.0 * tot_err.max() + 1e-6
    assert shaped >= 3, shaped


def pin_totals_planted(lib):
    """Per-depth totals against planted sources: noise-free single-pixel
    sources with integer amplitudes, one source per pixel, at four depths far
    apart.  The leading edge covers each source once during the scan, so the
    totals over the three bins around a depth hold exactly the summed
    amplitude of the sources at that depth, and every other bin holds none."""
    s = synth.tiny(40, 40, 61, 121, seed=51, step=1.0, width=1.0, n_src=48, dark=0.0,
                   noise=False, sigma=0.0, integer_amp=True, render_now=False)
    depths = np.array([-16.0, -5.5, 5.5, 16.0]) + 0.25
    src = s.sources
    n = len(src.zs)
    # one source per pixel, depths cycled over the four values
    rng = np.random.default_rng(52)
    flat = rng.choice(40 * 40, n, replace=False)
    src.ci[:] = (flat % 40).astype(np.float64)
    src.cj[:] = (flat // 40).astype(np.float64)
    src.zs[:] = depths[np.arange(n) % 4]
    synth.render(s)
    I = s.images.reshape(s.wire.n_steps, -1).astype(np.int64)
    out, tot, _ = oracle.reconstruct(s, lib=lib)
    e0 = s.grid.first_center - 0.5 * s.grid.width
    seen = np.zeros(s.grid.n_bins, dtype=bool)
    for z in depths:
        b = int(math.floor((z - e0) / s.grid.width))
        on = np.isclose(src.zs, z)
        # amplitude of the sources at this depth that the scan covers: the
        # count of the pixel drops by it once and never comes back
        covered = [int(src.amp[m]) for m in np.nonzero(on)[0]
                   if I[0, flat[m]] - I[-1, flat[m]] == int(src.amp[m])]
        assert len(covered) >= 8, (z, len(covered))
        want = float(sum(covered))
        got = float(tot[b - 1:b + 2].sum())
        assert abs(got - want) <= 1e-9 * want, (z, got, want)
        seen[b - 1:b + 2] = True
    # pixels without a source, or whose source is not covered, add nothing
    assert np.all(np.abs(tot[~seen]) <= 1e-9 * float(src.amp.sum())), tot[~seen]


def pin_planted_sources(lib):
    """Noise-free single-pixel sources with integer amplitude.  Leading edge:
    the source depth lies inside the interval of the step at which the pixel
    goes dark, and the bins of that interval receive exactly the amplitude.
    Trailing edge: the same for the step at which it comes back.  Both: the
    union of the two intervals' bins receives the amplitude (half from each)."""
    # long enough for the trailing edge (one shadow width, ~52 um, behind the
    # leading one) to pass the sources again before the scan ends
    s = synth.tiny(48, 48, 161, 161, seed=31, step=1.0, width=1.0, n_src=30, dark=0.0,
                   noise=False, sigma=0.0, integer_amp=True, zlo=-50.0, zhi=0.0)
    src = s.sources
    ii = np.rint(src.ci).astype(int)
    jj = np.rint(src.cj).astype(int)
    flat = jj * s.detector.nx + ii
    uniq, cnt = np.unique(flat, return_counts=True)
    single = set(uniq[cnt == 1].tolist())
    e0 = s.grid.first_center - 0.5 * s.grid.width
    B = s.grid.n_bins
    outs, ups = {}, {}
    for edge in (0, 1, 2):
        s.wire.edge = edge
        outs[edge], _, _ = oracle.reconstruct(s, lib=lib)
        _, _, ups[edge] = oracle.reconstruct_pixels(s, flat, want_u=True, lib=lib)

    def bins_of(u0, u1):
        b0 = max(0, int(math.floor(min(u0, u1))))
        b1 = min(B - 1, int(math.floor(max(u0, u1))))
        return set(range(b0, b1 + 1))

    checked = {0: 0, 1: 0, 2: 0}
    for n in range(len(flat)):
        if flat[n] not in single:
            continue
        I = s.images[:, jj[n], ii[n]].astype(np.int64)
        zu = (src.zs[n] - e0) / s.grid.width
        drops = np.nonzero(I[:-1] > I[1:])[0]
        rises = np.nonzero(I[:-1] < I[1:])[0]
        lead = trail = None
        if len(drops):
            k = int(drops[0])
            assert I[k] - I[k + 1] == int(src.amp[n])
            u0, u1 = ups[0][n, k], ups[0][n, k + 1]
            assert min(u0, u1) - 1e-9 <= zu <= max(u0, u1) + 1e-9, (zu, u0, u1)
            lead = bins_of(u0, u1)
            got = sum(outs[0][b, jj[n], ii[n]] for b in lead)
            assert abs(got - src.amp[n]) < 1e-8 * src.amp[n], (got, src.amp[n])
            checked[0] += 1
        if len(rises) and len(drops) and rises[-1] > drops[0]:
            k = int(rises[-1])
            assert I[k + 1] - I[k] == int(src.amp[n])
            u0, u1 = ups[1][n, k], ups[1][n, k + 1]
            assert min(u0, u1) - 1e-9 <= zu <= max(u0, u1) + 1e-9, (zu, u0, u1)
            trail = bins_of(u0, u1)
            got = sum(outs[1][b, jj[n], ii[n]] for b in trail)
            assert abs(got - src.amp[n]) < 1e-8 * src.amp[n], (got, src.amp[n])
            checked[1] += 1
        if lead is not None and trail is not None:
            got = sum(outs[2][b, jj[n], ii[n]] for b in (lead | trail))
            assert abs(got - src.amp[n]) < 1e-8 * src.amp[n], (got, src.amp[n])
            checked[2] += 1
    assert min(checked.values()) >= 8, checked


def pin_poisson_recovery(lib):
    """Poisson data: the +-1-bin smoothed profile of the brightest pixel of
    each clearly recoverable source peaks within one bin of its depth."""
    s = synth.tiny(160, 160, 81, 121, seed=41, step=1.0, width=1.0, n_src=120, dark=100.0,
                   noise=True, sigma=1.5)
    out, _, _ = oracle.reconstruct(s, lib=lib)
    src = s.sources
    e0 = s.grid.first_center - 0.5 * s.grid.width
    ii = np.rint(src.ci).astype(int)
    jj = np.rint(src.cj).astype(int)
    ok = tot = 0
    for n in range(len(src.zs)):
        # skip sources whose spots overlap another source's
        d = np.hypot(src.ci - src.ci[n], src.cj - src.cj[n])
        d[n] = np.inf
        if d.min() < 9.0:
            continue
        g = math.exp(-((ii[n] - src.ci[n]) ** 2 + (jj[n] - src.cj[n]) ** 2) / (2 * 1.5 ** 2))
        peak = src.amp[n] * g
        if peak < 20.0 * math.sqrt(peak + 100.0):
            continue
        prof = out[:, jj[n], ii[n]]
        sm = prof.copy()
        sm[1:] += prof[:-1]
        sm[:-1] += prof[1:]
        want = math.floor((src.zs[n] - e0) / s.grid.width)
        I = s.images[:, jj[n], ii[n]].astype(float)
        if I[:5].mean() - I.min() < 0.5 * peak:
            continue  # not occluded during the scan: not recoverable
        tot += 1
        ok += abs(int(np.argmax(sm)) - want) <= 1
    assert tot >= 30 and ok >= math.ceil(0.99 * tot), (ok, tot)


# ------------------------------------------------- tilted wire axis (3D pins)


def line_segment_dist3(C, a, S, P):
    """Distance between the line C + t*a (a unit) and the segment S->P in 3D,
    from the closest points of the two lines, the segment parameter clamped."""
    C, a, S, P = (np.asarray(x, dtype=np.float64) for x in (C, a, S, P))
    d = P - S
    w = S - C
    A, Bq, Cq = float(a @ a), float(a @ d), float(d @ d)
    D, E = float(a @ w), float(d @ w)
    den = A * Cq - Bq * Bq
    sp = (A * E * -1.0 + Bq * D) / den if den > 0 else 0.0
    sp = min(1.0, max(0.0, sp))
    t = (float(a @ (S + sp * d - C))) / A
    return float(np.linalg.norm(C + t * a - (S + sp * d)))


def random_tilted(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ax = np.array([1.0, rng.uniform(-0.4, 0.4), rng.uniform(-0.5, 0.5)])
        ax /= np.linalg.norm(ax)
        P = np.array([rng.uniform(-2e4, 2e4), rng.uniform(3e5, 6e5), rng.uniform(-2e5, 2e5)])
        C = np.array([rng.uniform(-500, 500), rng.uniform(100, 1500), rng.uniform(-300, 300)])
        r = rng.uniform(5.0, 60.0)
        out.append((ax, P, C, r))
    return out


def _oracle_positions(ax, P, centers, r, edge, lib):
    """u_k of one pixel at P (grid e0 = 0, width 1: u = depth)."""
    det = synth.Detector(1, 1, np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 0, 1.0]),
                         pixel_xyz=P.reshape(1, 1, 3))
    wire = synth.Wire(radius=r, centers=np.asarray(centers, dtype=np.float64), axis=ax, edge=edge)
    scan = synth.Scan("p", det, wire, synth.DepthGrid(4, 0.5, 1.0), None, 0.0, False, 0)
    _, _, u = oracle.reconstruct_pixels(scan, [0], want_bins=False, want_u=True, lib=lib)
    return u[0]


def pin_tilted_axis_bisection(lib):
    """A wire axis tilted out of x: the depth of each edge equals the beam point
    where the 3D distance between the axis line and the source-pixel segment
    reaches r, found by bisection (leading: downstream side for a wire moving
    downstream; trailing: upstream side)."""
    for ax, P, C, r in random_tilted(60, 16):
        step = np.array([0.0, 0.7, 0.7])
        centers = np.stack([C, C + step])
        dist = lambda z: line_segment_dist3(C, ax, np.array([0.0, 0.0, z]), P)
        # beam point whose ray meets the axis: minimise the distance
        lo, hi = -1e5, 1e5
        for _ in range(300):
            m1, m2 = lo + (hi - lo) / 3, hi - (hi - lo) / 3
            if dist(m1) < dist(m2):
                hi = m2
            else:
                lo = m1
        zc = 0.5 * (lo + hi)
        assert dist(zc) < r
        for edge, sgn in ((0, +1.0), (1, -1.0)):
            a_, b_ = zc, zc + sgn * 1e5
            for _ in range(200):
                m = 0.5 * (a_ + b_)
                if dist(m) < r:
                    a_ = m
                else:
                    b_ = m
            u = _oracle_positions(ax, P, centers, r, edge, lib)
            assert abs(u[0] - 0.5 * (a_ + b_)) < 1e-6 * (1 + abs(u[0])), (edge, u[0], a_, ax)


def pin_tilted_axis_brute_force(lib):
    """Tilted axis: whole-profile check against brute-force sub-sampling of the
    beam with the 3D occlusion predicate, arbitrary intensities."""
    rng = np.random.default_rng(17)
    for ax, P, C, r in random_tilted(4, 18):
        N = 7
        step = np.array([0.0, 0.8, 0.8])
        centers = np.stack([C + (k - N // 2) * step for k in range(N)])
        # grid around the leading sweep
        u0 = _oracle_positions(ax, P, centers, r, 0, lib)
        width = 0.5
        B = 40
        first = np.floor(u0.min()) - 8.0
        det = synth.Detector(1, 1, np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 0, 1.0]),
                             pixel_xyz=P.reshape(1, 1, 3))
        I = rng.integers(0, 60000, N).astype(np.uint16)
        for edge in (0, 1, 2):
            wire = synth.Wire(radius=r, centers=centers, axis=ax, edge=edge)
            grid = synth.DepthGrid(B, first + 0.5 * width, width)
            scan = synth.Scan("bf", det, wire, grid, None, 0.0, False, 0,
                              images=I.reshape(N, 1, 1))
            out, _, _ = oracle.reconstruct(scan, lib=lib)
            e0 = first
            h = width / 2500.0
            z = e0 - 40.0 * width + h * (np.arange(int((B + 80) * width / h)) + 0.5)
            # vectorised 3D distance: closest points between the axis line and each segment
            dvec = P[None, :] - np.stack([np.zeros_like(z), np.zeros_like(z), z], 1)
            prof = {0: np.zeros(B), 1: np.zeros(B)}
            err = {0: np.zeros(B), 1: np.zeros(B)}
            occ = []
            for c in centers:
                S = np.stack([np.zeros_like(z), np.zeros_like(z), z], 1)
                w = S - c[None, :]
                A = 1.0
                Bq = dvec @ ax
                Cq = np.einsum("ij,ij->i", dvec, dvec)
                D = w @ ax
                E = np.einsum("ij,ij->i", dvec, w)
                sp = np.clip((Bq * D - A * E) / (A * Cq - Bq * Bq), 0.0, 1.0)
                Q = S + sp[:, None] * dvec
                t = (Q - c[None, :]) @ ax
                occ.append(np.linalg.norm(c[None, :] + t[:, None] * ax[None, :] - Q, axis=1) < r)
            occ = np.stack(occ)
            binidx = np.floor((z - e0) / width).astype(np.int64)
            inside = (binidx >= 0) & (binidx < B)
            for side in (0, 1):
                for k in range(N - 1):
                    newly = (occ[k + 1] & ~occ[k]) if side == 0 else (occ[k] & ~occ[k + 1])
                    dI = (float(I[k]) - float(I[k + 1])) * (1 if side == 0 else -1)
                    n = int(newly.sum())
                    if n == 0:
                        continue
                    cnt = np.bincount(binidx[newly & inside], minlength=B)
                    prof[side] += dI * cnt / n
                    err[side][cnt > 0] += abs(dI) * 4.0 / n
            want = prof[0] if edge == 0 else (prof[1] if edge == 1 else 0.5 * (prof[0] + prof[1]))
            tol = err[0] if edge == 0 else (err[1] if edge == 1 else 0.5 * (err[0] + err[1]))
            assert np.all(np.abs(out[:, 0, 0] - want) <= tol + 1e-6), (edge, ax)



def pin_activity(lib):
    """Pixel activity sum_k |I_k - I_{k+1}|: a monotone series gives
    |I_last - I_first|; a constant series 0; a sawtooth of height h over N
    samples (N-1)*h, beyond 32 bits for a long full-range sawtooth; reversing
    the steps or adding an offset leaves it unchanged."""
    rng = np.random.default_rng(41)
    N, npix = 37, 50
    inc = np.sort(rng.integers(0, 60000, (N, npix)), axis=0).astype(np.uint16)
    dec = inc[::-1].copy()
    a_inc = oracle.activity(inc, lib=lib)
    a_dec = oracle.activity(dec, lib=lib)
    expect = inc[-1].astype(np.uint64) - inc[0].astype(np.uint64)
    assert np.array_equal(a_inc, expect) and np.array_equal(a_dec, expect)
    const = np.full((N, 3), 1234, dtype=np.uint16)
    assert np.all(oracle.activity(const, lib=lib) == 0)
    n_long = 70001
    saw = np.zeros((n_long, 2), dtype=np.uint16)
    saw[1::2, 0] = 65535
    saw[1::2, 1] = 7
    a = oracle.activity(saw, lib=lib)
    assert int(a[0]) == (n_long - 1) * 65535 and int(a[1]) == (n_long - 1) * 7
    noisy = rng.integers(0, 30000, (N, npix)).astype(np.uint16)
    a0 = oracle.activity(noisy, lib=lib)
    assert np.array_equal(oracle.activity(noisy[::-1].copy(), lib=lib), a0)
    assert np.array_equal(oracle.activity(noisy + np.uint16(20000), lib=lib), a0)


def pin_select_top(lib):
    """Top-k selection: k entries in increasing index order such that every
    selected pixel ranks before every unselected one (larger activity, or
    equal activity and lower index); k = 0 and k = n are the empty and full
    lists."""
    rng = np.random.default_rng(42)
    for n, hi in ((1, 3), (17, 4), (200, 6), (1000, 1000)):
        act = rng.integers(0, hi, n).astype(np.uint64)
        for k in sorted({0, 1, n // 3, n // 2, n - 1, n} - {-1}):
            if k < 0:
                continue
            sel = oracle.select_top(act, k, lib=lib)
            assert sel.shape == (k,)
            assert np.all(np.diff(sel) > 0)
            if k in (0, n):
                assert np.array_equal(sel, np.arange(k))
            chosen = np.zeros(n, dtype=bool)
            chosen[sel] = True
            if 0 < k < n:
                p = np.nonzero(chosen)[0]
                q = np.nonzero(~chosen)[0]
                ap, aq = act[p][:, None], act[q][None, :]
                ranks_before = (ap > aq) | ((ap == aq) & (p[:, None] < q[None, :]))
                assert ranks_before.all(), (n, k)


def pin_step_weights(lib):
    """Per-step weights (monitor normalisation): a stack whose images were
    multiplied by monitor factors m_k in {1, 2}, weighted by 1/m_k, gives the
    unmodulated reconstruction bit for bit (and the unweighted modulated one
    differs); weights of 4 scale the output by exactly 4; with arbitrary
    weights each pixel whose sweep lies inside the grid conserves
    I_0 w_0 - I_{N-1} w_{N-1}."""
    base = synth.tiny(24, 3, 21, 61, seed=61, n_src=5, dark=50.0, noise=False)
    base.images = (base.images // 2).astype(np.uint16)
    base.grid = synth.DepthGrid(100, -74.5, 1.0)  # holds the sweeps of both edges
    rng = np.random.default_rng(61)
    m = rng.integers(1, 3, base.wire.n_steps).astype(np.float64)
    modulated = (base.images.astype(np.int64) * m[:, None, None].astype(np.int64)).astype(np.uint16)
    for edge in (0, 1, 2):
        w0 = synth.Wire(base.wire.radius, base.wire.centers, edge=edge)
        plain = synth.Scan("p", base.detector, w0, base.grid, None, 0.0, False, 0,
                           images=base.images)
        ref, _, _ = oracle.reconstruct(plain, lib=lib)
        ww = synth.Wire(base.wire.radius, base.wire.centers, edge=edge, weights=1.0 / m)
        norm = synth.Scan("n", base.detector, ww, base.grid, None, 0.0, False, 0,
                          images=modulated)
        got, _, _ = oracle.reconstruct(norm, lib=lib)
        assert np.array_equal(got, ref), edge
        raw, _, _ = oracle.reconstruct(synth.Scan("r", base.detector, w0, base.grid, None, 0.0,
                                                  False, 0, images=modulated), lib=lib)
        assert not np.array_equal(raw, ref)
        pix = np.arange(24 * 3)
        gp, _, _ = oracle.reconstruct_pixels(norm, pix, want_bins=False, lib=lib)
        assert np.array_equal(gp.T.reshape(ref.shape), ref), edge
        w4 = synth.Wire(base.wire.radius, base.wire.centers, edge=edge,
                        weights=np.full(base.wire.n_steps, 4.0))
        g4, _, _ = oracle.reconstruct(synth.Scan("4", base.detector, w4, base.grid, None, 0.0,
                                                 False, 0, images=base.images), lib=lib)
        assert np.array_equal(g4, 4.0 * ref), edge
    wr = rng.uniform(0.5, 2.0, base.wire.n_steps)
    sc = synth.Scan("w", base.detector, synth.Wire(base.wire.radius, base.wire.centers,
                                                   weights=wr),
                    base.grid, None, 0.0, False, 0, images=base.images)
    out, _, bins = oracle.reconstruct(sc, want_bins=True, lib=lib)
    I = base.images.reshape(base.wire.n_steps, -1).astype(np.float64)
    want = I[0] * wr[0] - I[-1] * wr[-1]
    inside = (bins.min(1) >= 0) & (bins.max(1) <= base.grid.n_bins - 1)
    assert inside.sum() > 10
    sums = out.reshape(base.grid.n_bins, -1).sum(0)
    assert np.allclose(sums[inside], want[inside], rtol=0, atol=1e-9 * np.abs(I).sum(0).max())

ALL_PINS = [
    pin_closed_form_level, pin_zero_radius, pin_bisection, pin_mirror, pin_edge_sign,
    pin_hand_profiles, pin_conservation_random, pin_conservation_scan, pin_brute_force,
    pin_totals_planted, pin_planted_sources, pin_poisson_recovery, pin_tilted_axis_bisection,
    pin_tilted_axis_brute_force, pin_activity, pin_select_top, pin_step_weights,
]
