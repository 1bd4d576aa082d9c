"""Pins of the oracle's pyramid and histogram rule (Sec. 3.4, Algorithm 1)
against closed forms, invariants and analytic scenes.  CPU only."""
import os

import numpy as np
import pytest

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _plane_table():
    rows = []
    with open(os.path.join(GOLDEN, "plane_bins.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            d, r0, r1 = line.split()
            rows.append((int(d), None if r0 == "-" else int(r0), None if r1 == "-" else int(r1)))
    return rows


# ---------------------------------------------------------------------------
# pyramid
# ---------------------------------------------------------------------------
def test_pyramid_sizes_and_levels():
    for W, H in [(1, 1), (2, 1), (5, 3), (128, 128), (1024, 768), (7, 1)]:
        L = oracle.pyr_levels(W, H)
        sizes = []
        w, h = W, H
        while True:
            sizes.append(w * h)
            if w == 1 and h == 1:
                break
            w, h = -(-w // 2), -(-h // 2)
        assert L == len(sizes)
        assert oracle.pyr_floats(W, H) == sum(sizes)


def test_pyramid_block_means_integer_maps():
    # integer depths: sums of up to 4^l integers are exact in float32 and the
    # level-l pixel is the mean of its 2^l x 2^l block (equal child counts)
    rng = np.random.default_rng(0)
    d = rng.integers(1, 64, size=(32, 16)).astype(np.float32)
    levels = oracle.pyramid_levels(oracle.pyramid(d), 16, 32)
    for l, lev in enumerate(levels):
        b = 2 ** l
        bh, bw = max(1, 32 // b), max(1, 16 // b)
        if 32 % b or 16 % b:
            continue
        blocks = d.astype(np.float64).reshape(bh, b, bw, b).mean(axis=(1, 3))
        # means of means of four: exact while the partial sums stay integral /4^m
        np.testing.assert_allclose(lev, blocks, rtol=2e-7)


def test_pyramid_invalid_children_and_constant_map():
    d = np.full((8, 8), 3.5, dtype=np.float32)
    d[0, 0] = np.nan
    d[0, 1] = -1.0
    d[1, 0] = np.inf
    d[1, 1] = 0.0
    levels = oracle.pyramid_levels(oracle.pyramid(d), 8, 8)
    assert levels[0][0, 0] == 0 and levels[0][0, 1] == 0 and levels[0][1, 0] == 0
    assert levels[1][0, 0] == 0.0          # all four children invalid
    assert levels[1][0, 1] == np.float32(3.5)
    assert levels[2][0, 0] == np.float32(3.5)  # invalid children are skipped, not averaged in
    assert levels[-1].shape == (1, 1) and levels[-1][0, 0] == np.float32(3.5)
    d2 = np.zeros((4, 4), dtype=np.float32)
    d2[3, 3] = 2.0
    d2[0, 0] = 4.0
    lv = oracle.pyramid_levels(oracle.pyramid(d2), 4, 4)
    assert lv[1][1, 1] == 2.0 and lv[1][0, 0] == 4.0 and lv[2][0, 0] == 3.0


def test_pyramid_odd_sizes_every_pixel_has_a_parent():
    d = np.arange(1, 1 + 5 * 3, dtype=np.float32).reshape(3, 5)
    lv = oracle.pyramid_levels(oracle.pyramid(d), 5, 3)
    assert lv[1].shape == (2, 3)
    # last column of level 1 has only children (4, 0) and (4, 1)
    assert lv[1][0, 2] == np.float32((d[0, 4] + d[1, 4]) / 2)
    # bottom-right parent has a single child
    assert lv[1][1, 2] == d[2, 4]


# ---------------------------------------------------------------------------
# histogram rule on an analytic plane
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rule", [0, 1])
def test_plane_bins_match_golden_table(rule):
    table = _plane_table()
    zi = 12
    sc = scenes.plane_scene(n=(3, 3, 28), z_plane_index=zi, n_cams=1)
    hist, _ = oracle.histograms(sc, rule=rule)
    H = hist.reshape(28, 3, 3, 8)[:, 1, 1, :]
    for d, b0, b1 in table:
        k = zi - d
        expected = b0 if rule == 0 else b1
        row = H[k]
        if expected is None:
            assert row.sum() == 0, (d, row)
        else:
            assert row[expected] == 1 and row.sum() == 1, (d, row)


def test_plane_votes_add_over_cameras_with_weights():
    sc = scenes.plane_scene(n=(4, 3, 10), z_plane_index=4, n_cams=4)
    sc.cams.vote[:] = [1, 5, 1, 5]
    hist, mx = oracle.histograms(sc)
    H = hist.reshape(10, 3, 4, 8)
    assert mx == 12
    for k in range(10):
        d = 4 - k
        b = min(6, max(0, 3 + d))
        assert H[k, 1, 1, b] == 12 and H[k, 1, 1].sum() == 12


def test_mip_level_selection_reads_coarser_level():
    # voxel h = 0.25 at camera depth 4 with fx = 64 projects to s = 4 pixels:
    # level floor(log2 4) = 2 must be read.  The map alternates two depths on
    # a 2x2 checker (levels >= 1 hold their mean), so reading level 0 would
    # give a different bin.
    sc = scenes.plane_scene(n=(1, 1, 9), z_plane_index=4, n_cams=1, distance=4.0, f=64.0, W=64, H=64)
    near, far = 4.0 - 0.75, 4.0 + 0.75  # level-0 samples: +-3 voxels (bins 6 / 0)
    yy, xx = np.mgrid[0:64, 0:64]
    d = np.where(((xx // 1) + (yy // 1)) % 2 == 0, near, far).astype(np.float32)
    sc.depth[0] = d
    hist, _ = oracle.histograms(sc)
    H = hist.reshape(9, 8)
    # level-2 sample is the mean 4.0, so the voxel on the plane gets bin 3
    assert H[4, 3] == 1, H[4]
    # a camera much closer: s < 1 picks level 0, whose pixel reads near or far
    sc2 = scenes.plane_scene(n=(1, 1, 9), z_plane_index=4, n_cams=1, distance=4.0, f=8.0, W=64, H=64)
    sc2.depth[0] = d
    H2 = oracle.histograms(sc2)[0].reshape(9, 8)
    assert H2[4, 3] == 0 and H2[4].sum() == 1


def test_no_vote_outside_image_behind_camera_or_invalid():
    sc = scenes.plane_scene(n=(3, 3, 5), z_plane_index=2, n_cams=1, distance=20.0)
    # move the camera sideways so the block leaves the image
    sc.cams.t[0, 0] += 1000.0
    assert oracle.histograms(sc)[0].sum() == 0
    sc = scenes.plane_scene(n=(3, 3, 5), z_plane_index=2, n_cams=1, distance=20.0)
    sc.cams.t[0, 2] -= 100.0  # block now behind the camera
    assert oracle.histograms(sc)[0].sum() == 0
    sc = scenes.plane_scene(n=(3, 3, 5), z_plane_index=2, n_cams=1, distance=20.0)
    sc.depth[:] = np.nan
    assert oracle.histograms(sc)[0].sum() == 0


# ---------------------------------------------------------------------------
# invariants on the sphere scene
# ---------------------------------------------------------------------------
def test_sphere_histograms_invariants():
    sc = scenes.sphere_scene(n=16)
    pyr = oracle.pyramids(sc.depth)
    full, mx = oracle.histograms(sc, pyr)
    assert mx <= int(sc.cams.vote.sum())
    assert full[:, 7].sum() == 0
    # additivity over cameras (so culling a camera that casts no vote and the
    # camera order cannot change a count)
    acc = np.zeros_like(full, dtype=np.int64)
    for k in range(len(sc.cams)):
        sub = scenes.Scene(sc.depth[k:k + 1], sc.cams.subset([k]), sc.grid)
        acc += oracle.histograms(sub)[0]
    np.testing.assert_array_equal(acc, full)
    perm = np.random.default_rng(3).permutation(len(sc.cams))
    sp = scenes.Scene(sc.depth[perm], sc.cams.subset(perm), sc.grid)
    np.testing.assert_array_equal(oracle.histograms(sp)[0], full)
    # a selection of voxels equals the same rows of the full pass
    sel = np.array([0, 5, 100, 2047, 4095])
    np.testing.assert_array_equal(oracle.histograms(sc, pyr, vox=sel)[0], full[sel])


def test_threaded_histograms_equal_serial():
    sc = scenes.sphere_scene(n=20)
    pyr = oracle.pyramids(sc.depth)
    ref, mx = oracle.histograms(sc, pyr)
    with oracle.threads(4):
        got, mx4 = oracle.histograms(sc, pyr)
    np.testing.assert_array_equal(got, ref)
    assert mx4 == mx


def test_sphere_noise_free_geometry():
    sc = scenes.sphere_scene(n=64, sigma=0.0, outlier_frac=0.0)
    hist, _ = oracle.histograms(sc)
    g = sc.grid
    idx = np.arange(g.nvox)
    i, j, k = idx % 64, (idx // 64) % 64, idx // 4096
    P = g.origin.astype(np.float64) + (np.stack([i, j, k], 1) + 0.5) * g.h
    r = np.linalg.norm(P, axis=1)
    h = g.h
    # deep inside the sphere (more than eta = 9 voxels behind every visible
    # surface point along the ray plus a pixel footprint): no votes at all
    deep = r < 1.0 - 9.0 * h - 0.1
    assert deep.any() and hist[deep].sum() == 0
    # every vote cast on a voxel more than delta + footprint outside the sphere
    # is a free-space vote (bin 6)
    outside = r > 1.0 + 3.0 * h + 0.1
    assert hist[outside, :6].sum() == 0 and hist[outside, 6].sum() > 0
    # voxels on the surface shell get near-surface votes (bins 2..4) from the
    # cameras that see them from the front; cameras behind the sphere see
    # them as occluded (bin 0 or no vote), never as free space
    shell = np.abs(r - 1.0) < 0.25 * h
    assert (hist[shell][:, 2:5].sum(1) > 0).mean() > 0.9
    assert hist[shell][:, 6].sum() < 0.05 * hist[shell].sum()


def test_sphere_generator_depth_on_surface():
    sc = scenes.sphere_scene(sigma=0.0, outlier_frac=0.0)
    for kc in range(len(sc.cams)):
        C, d = scenes.pixel_rays(sc.cams, kc)
        z = scenes.sphere_depth(sc.cams, kc)
        P = C[None, None, :] + z[..., None] * d
        hit = z > 0
        np.testing.assert_allclose(np.linalg.norm(P[hit], axis=1), 1.0, atol=1e-12)
        # rays that miss pass the origin at a distance > 1
        dn = d / np.linalg.norm(d, axis=-1, keepdims=True)
        closest = np.linalg.norm(np.cross(dn, -C[None, None, :]), axis=-1)
        assert np.all(closest[~hit] > 1.0 - 1e-12)
        assert np.array_equal(sc.depth[kc] > 0, hit)


def test_scene_seeds_reproduce():
    a = scenes.sphere_scene(seed=7)
    b = scenes.sphere_scene(seed=7)
    c = scenes.sphere_scene(seed=8)
    assert a.digest() == b.digest() and a.digest() != c.digest()
    t1 = scenes.terrain_scene(n=32, n_side=2, W=64, H=64, f=96.0, lattice=128)
    t2 = scenes.terrain_scene(n=32, n_side=2, W=64, H=64, f=96.0, lattice=128)
    assert t1.digest() == t2.digest()
    assert (t1.depth > 0).mean() > 0.99


# ---------------------------------------------------------------------------
# 360-degree scans (Sec. 3.1: terrestrial LIDAR as 360-degree depth maps,
# vote 5 in Algorithm 1) as equirectangular range maps
# ---------------------------------------------------------------------------
def test_scan_pixel_of_axis_directions():
    """The axis directions land on the quadrant and equator boundaries:
    +x column 0, +y W/4, -x W/2, -y 3W/4 (all on row H/2, the equator's
    row); +z row 0 and -z row H-1."""
    W, H = 64, 32
    tab = oracle.scan_tables(W, H)
    assert oracle.scan_pixel(1, 0, 0, 1, W, H, tab) == (0, H // 2)
    assert oracle.scan_pixel(0, 1, 0, 1, W, H, tab) == (W // 4, H // 2)
    assert oracle.scan_pixel(-1, 0, 0, 1, W, H, tab) == (W // 2, H // 2)
    assert oracle.scan_pixel(0, -1, 0, 1, W, H, tab) == (3 * W // 4, H // 2)
    assert oracle.scan_pixel(0, 0, 1, 1, W, H, tab)[1] == 0
    assert oracle.scan_pixel(0, 0, -1, 1, W, H, tab)[1] == H - 1
    C, S, K = tab
    assert C[0] == 1.0 and S[0] == 0.0 and K[0] == 1.0
    assert (np.diff(C) <= 0).all() and (np.diff(S) >= 0).all() and (np.diff(K) <= 0).all()
    # a direction exactly on a boundary belongs to the pixel that boundary
    # opens (pixels are half-open): column i for (C_i, S_i) in every
    # quadrant, row j where z equals K_j times the range exactly
    for i in (1, 5, W // 4 - 1):
        for q, (x, y) in enumerate([(C[i], S[i]), (-S[i], C[i]), (-C[i], -S[i]), (S[i], -C[i])]):
            assert oracle.scan_pixel(x, y, 0.0, 1.0, W, H, tab)[0] == q * W // 4 + i, (i, q)
    on_row = 0
    for j in range(1, H):
        z = np.float32(K[j])
        x = np.float32(np.sqrt(max(0.0, 1.0 - float(z) * float(z))))
        rho = np.float32(np.sqrt(np.float32(np.float32(x * x) + np.float32(z * z))))
        if rho == np.float32(1.0):
            assert oracle.scan_pixel(x, 0.0, z, rho, W, H, tab)[1] == j, j
            on_row += 1
    assert on_row >= 3


@pytest.mark.parametrize("W,H", [(64, 32), (2048, 1024), (12, 5)])
def test_scan_pixel_matches_float64_angles(W, H):
    """Away from a pixel boundary, the sign-test pixel equals the textbook
    equirectangular pixel floor(phi W / 2 pi), floor(theta H / pi) with phi =
    atan2(y, x) in [0, 2 pi) and theta = acos(z / |d|) taken in float64."""
    rng = np.random.default_rng(W + H)
    d = rng.normal(size=(4000, 3)).astype(np.float32)
    d[:200, 2] = 0.0  # on the equator
    d[200:300, :2] *= 1e-3  # near the poles
    tab = oracle.scan_tables(W, H)
    checked = 0
    for x, y, z in d:
        x64, y64, z64 = float(x), float(y), float(z)
        rho32 = np.float32(np.sqrt(np.float32(np.float32(x * x) + np.float32(y * y)) + np.float32(z * z)))
        phi = np.arctan2(y64, x64) % (2 * np.pi)
        theta = np.arccos(z64 / np.sqrt(x64 * x64 + y64 * y64 + z64 * z64))
        fc, fr = phi * W / (2 * np.pi), theta * H / np.pi
        if min(fc % 1.0, 1 - fc % 1.0) < 1e-3 or min(fr % 1.0, 1 - fr % 1.0) < 1e-3:
            continue
        col, row = oracle.scan_pixel(x, y, z, rho32, W, H, tab)
        assert (col, row) == (int(fc) % W, int(fr)), (x, y, z)
        checked += 1
    assert checked > 3000


def _scanner_in_sphere(m=16, n=61, W=64, H=32):
    """A scanner at the centre voxel of an n^3 block (h = 1/16) inside a
    sphere of radius m h centred on it: a noise-free constant range map."""
    h = 1.0 / 16
    c = n // 2
    origin = np.full(3, -(c + 0.5) * h, dtype=np.float32)
    cams = scenes.scan360_cameras([(0.0, 0.0, 0.0)], W, H)
    depth = np.full((1, H, W), np.float32(m * h), dtype=np.float32)
    return scenes.Scene(depth, cams, scenes.Grid(origin, h, (n, n, n), 0)), c


def test_scan_inside_sphere_bins_by_range_golden():
    """Voxels on the six axes through the scanner lie at range k h exactly;
    with the surface at range m h they are d = m - k voxels in front of it
    and bin as the fronto-parallel plane's golden table says (the scan's
    distance is the range, the same delta = 3 voxels and eta = 9)."""
    m = 16
    sc, c = _scanner_in_sphere(m)
    n = sc.grid.n[0]
    hist, _ = oracle.histograms(sc)
    Hh = hist.reshape(n, n, n, 8)
    table = {d: b0 for d, b0, _ in _plane_table()}
    seen = 0
    for axis in range(3):
        for sign in (1, -1):
            for k in range(1, c + 1):
                idx = [c, c, c]
                idx[axis] += sign * k
                row = Hh[idx[2], idx[1], idx[0]]
                d = m - k
                if d not in table:
                    continue
                expected = table[d]
                if expected is None:
                    assert row.sum() == 0, (axis, sign, k, row)
                else:
                    assert row[expected] == 5 and row.sum() == 5, (axis, sign, k, row)
                seen += 1
    assert seen == 6 * 13
    assert Hh[c, c, c].sum() == 0  # the scanner's own voxel has no direction


def test_mixed_sizes_and_models_add_up():
    """Pinhole maps of 128^2 and a 512 x 256 scan in one histogram call
    equal the sum of their separate calls (each camera reads its own
    pyramid at its own size)."""
    ring = scenes.sphere_scene(n=24)
    scan = scenes.scan360_sphere_scene(n=24)
    cams = scenes.concat_cameras(scan.cams, ring.cams)
    pyr = np.concatenate([oracle.pyramids(scan.depth), oracle.pyramids(ring.depth)])
    both, _ = oracle.histograms(scenes.Scene(None, cams, ring.grid), pyr)
    a, _ = oracle.histograms(scenes.Scene(ring.depth, ring.cams, ring.grid))
    b, _ = oracle.histograms(scenes.Scene(scan.depth, scan.cams, ring.grid))
    assert b.sum() > 0 and a.sum() > 0
    assert np.array_equal(both.astype(np.int64), a.astype(np.int64) + b.astype(np.int64))


def test_scan360_generator_geometry():
    """A scanner at a sphere's centre sees the radius in every pixel; a
    terrain scanner sees the ground `height` below it straight down and
    nothing above the horizon."""
    cams = scenes.scan360_cameras([(0.1, -0.2, 0.3)], 16, 8)
    r = scenes.sphere_range(cams, 0, radius=2.0, center=(0.1, -0.2, 0.3))
    np.testing.assert_allclose(r, 2.0, rtol=1e-7)  # the centre is kept in float32
    d, tc = scenes.terrain_scans360(positions=((0.4, 0.6),), W=64, H=32, n=32, sigma_vox=0.0)
    assert d.shape == (1, 32, 64) and list(tc.model) == [1] and list(tc.vote) == [5]
    assert (d[0, : 32 // 2 - 1] == 0).all()  # rows above the horizon
    assert abs(float(d[0, -1].mean()) - 0.03) < 2e-3  # the row around -z
