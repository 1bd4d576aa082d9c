"""360-degree scans (Sec. 3.1, Algorithm 1 with vote 5) as equirectangular
range maps, and cameras of different sizes in one histogram call: GPU
histograms against the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    return tgv.Context(0)


def _gpu_hist(ctx, depths, cams, grid, **kw):
    import paper_2107_14790_amd as tgv
    pyr, offs = ctx.build_pyramids_mixed([torch.from_numpy(d).cuda() for d in depths])
    h = ctx.build_histograms_ex(pyr, offs, cams, tgv.grid_from(grid), **kw)
    torch.cuda.synchronize()
    return h.cpu().numpy().view(np.uint16)


def test_scanner_inside_sphere_matches_oracle(ctx):
    """The pin scene: a scanner at a voxel centre inside a sphere of
    constant range; every voxel of the 61^3 block."""
    h = 1.0 / 16
    n, c, m = 61, 30, 16
    origin = np.full(3, -(c + 0.5) * h, dtype=np.float32)
    cams = scenes.scan360_cameras([(0.0, 0.0, 0.0)], 64, 32)
    depth = np.full((1, 32, 64), np.float32(m * h), dtype=np.float32)
    grid = scenes.Grid(origin, h, (n, n, n), 0)
    ref, _ = oracle.histograms(scenes.Scene(depth, cams, grid))
    got = _gpu_hist(ctx, [depth], cams, grid)
    assert ref.sum() > 0
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("W,H", [(512, 256), (4096, 2048), (12, 7)])
def test_scan_sphere_matches_oracle(ctx, W, H):
    """One scanner outside the unit sphere, noisy ranges, at several
    resolutions (down to 3 columns per quadrant)."""
    sc = scenes.scan360_sphere_scene(W=W, H=H, n=32)
    ref, _ = oracle.histograms(sc)
    got = _gpu_hist(ctx, [sc.depth], sc.cams, sc.grid)
    assert ref.sum() > 0
    assert np.array_equal(got, ref)


def test_mixed_sizes_in_one_call_match_oracle(ctx):
    """Eight 128^2 ring cameras and a 512 x 256 scan in one call; also the
    ring cameras through the single-size entry point."""
    import paper_2107_14790_amd as tgv
    ring = scenes.sphere_scene(n=32)
    scan = scenes.scan360_sphere_scene(n=32)
    cams = scenes.concat_cameras(ring.cams, scan.cams)
    pyr = np.concatenate([oracle.pyramids(ring.depth), oracle.pyramids(scan.depth)])
    ref, _ = oracle.histograms(scenes.Scene(None, cams, ring.grid), pyr)
    got = _gpu_hist(ctx, [ring.depth, scan.depth], cams, ring.grid)
    assert np.array_equal(got, ref)
    # the same cameras with the scan listed first
    cams2 = scenes.concat_cameras(scan.cams, ring.cams)
    got2 = _gpu_hist(ctx, [scan.depth, ring.depth], cams2, ring.grid)
    assert np.array_equal(got2, ref)
    # single-size entry point (all ring maps 128^2) against the oracle
    p = ctx.build_pyramids(torch.from_numpy(ring.depth).cuda())
    h1 = ctx.build_histograms(p, 128, 128, ring.cams, tgv.grid_from(ring.grid)).cpu().numpy().view(np.uint16)
    assert np.array_equal(h1, oracle.histograms(ring)[0])


def test_accumulate_across_calls_equals_one_call(ctx):
    """Stereo maps in one call, the scan added in a second call with
    TGV_HIST_ACCUMULATE: the same counts as one call with both."""
    import paper_2107_14790_amd as tgv
    ring = scenes.sphere_scene(n=32)
    scan = scenes.scan360_sphere_scene(n=32)
    g = tgv.grid_from(ring.grid)
    pr, orr = ctx.build_pyramids_mixed([torch.from_numpy(ring.depth).cuda()])
    ps, osc = ctx.build_pyramids_mixed([torch.from_numpy(scan.depth).cuda()])
    h = ctx.build_histograms_ex(pr, orr, ring.cams, g)
    ctx.build_histograms_ex(ps, osc, scan.cams, g, accumulate=True, prior_votes=8, out=h)
    torch.cuda.synchronize()
    both = _gpu_hist(ctx, [ring.depth, scan.depth], scenes.concat_cameras(ring.cams, scan.cams), ring.grid)
    assert np.array_equal(h.cpu().numpy().view(np.uint16), both)


def test_histogram_errors(ctx):
    import paper_2107_14790_amd as tgv
    scan = scenes.scan360_sphere_scene(n=16)
    g = tgv.grid_from(scan.grid)
    pyr, offs = ctx.build_pyramids_mixed([torch.from_numpy(scan.depth).cuda()])
    h = ctx.build_histograms_ex(pyr, offs, scan.cams, g)
    with pytest.raises(tgv.TgvError) as e:  # 65535 prior votes + 5
        ctx.build_histograms_ex(pyr, offs, scan.cams, g, accumulate=True, prior_votes=65535, out=h)
    assert e.value.status == tgv.TGV_E_OVERFLOW
    bad = scan.cams.subset([0])
    bad.wh[0, 0] = 510  # not divisible by 4
    with pytest.raises(tgv.TgvError) as e:
        ctx.build_histograms_ex(pyr, offs, bad, g)
    assert e.value.status == tgv.TGV_E_INVAL
    bad = scan.cams.subset([0])
    bad.model[0] = 7
    with pytest.raises(tgv.TgvError) as e:
        ctx.build_histograms_ex(pyr, offs, bad, g)
    assert e.value.status == tgv.TGV_E_INVAL
    with pytest.raises(tgv.TgvError) as e:  # prior votes without accumulating
        ctx.build_histograms_ex(pyr, offs, scan.cams, g, prior_votes=3)
    assert e.value.status == tgv.TGV_E_INVAL
