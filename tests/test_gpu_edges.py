"""Degenerate inputs through the C ABI: no cameras, no blocks, no
iterations beyond the first, fields without a zero level, and a camera that
sees none of the block.  Each is checked against what the definition (or
the oracle) gives."""
import sys

import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[edge]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    c = tgv.Context(0)
    yield c
    c.close()


def test_no_cameras_gives_empty_histograms(ctx):
    import paper_2107_14790_amd as tgv
    say("no cameras")
    sc = scenes.sphere_scene(n=16)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    hist = torch.full((16 ** 3, 8), 7, dtype=torch.int16, device="cuda")
    ctx.build_histograms(pyr, W, H, sc.cams.subset([]), tgv.grid_from(sc.grid), out=hist)
    assert not hist.any()


def test_camera_that_sees_nothing_is_culled_and_votes_nothing(ctx):
    import paper_2107_14790_amd as tgv
    say("camera looking away")
    sc = scenes.sphere_scene(n=16)
    # the first ring camera turned around: it looks away from the block
    cams = sc.cams.subset([0])
    cams.R[0] = -cams.R[0] * np.array([[1], [-1], [1]], dtype=np.float32)  # still a rotation
    cams.t[0] = -(cams.R[0] @ sc.cams.centers()[0]).astype(np.float32)
    assert len(ctx.cull(cams, tgv.grid_from(sc.grid))) == 0
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth[:1]).cuda())
    hist = ctx.build_histograms(pyr, W, H, cams, tgv.grid_from(sc.grid))
    assert not hist.any()
    ref, _ = oracle.histograms(scenes.Scene(sc.depth[:1], cams, sc.grid))
    assert not ref.any()


def test_empty_batch_and_zero_iterations(ctx):
    import paper_2107_14790_amd as tgv
    say("empty batch, zero iterations")
    ctx.solve_batch([], [], tgv.Params(iters=10))
    g = tgv.grid_c((0, 0, 0), 1.0, (9, 8, 7), 1)
    st = tgv.State(ctx, g)
    u0 = torch.linspace(-1, 1, 9 * 8 * 7, device="cuda")
    st.reset(u0)
    hist = torch.zeros((9 * 8 * 7, 8), dtype=torch.int16, device="cuda")
    ctx.solve_batch([st], [hist], tgv.Params(iters=0))
    assert torch.equal(st.export()["u"], u0)
    st.close()


@pytest.mark.parametrize("iters", [1, 2, 3])
def test_first_iterations_match_oracle(ctx, iters):
    """1 iteration (dual and primal steps only), 2 (one fused pass) and 3
    (one two-iteration pass) on a block that takes the two-iteration kernel."""
    import paper_2107_14790_amd as tgv
    say("first iterations", iters)
    shape = (70, 30, 18)
    rng = np.random.default_rng(iters)
    n = int(np.prod(shape))
    hist = np.zeros((n, 8), dtype=np.uint16)
    hist[:, :7] = rng.integers(0, 4, size=(n, 7))
    u0 = rng.uniform(-1, 1, n).astype(np.float32)
    g = tgv.grid_c((0, 0, 0), 1.0, shape, 1)
    u = torch.from_numpy(u0).cuda()
    ctx.solve(g, torch.from_numpy(hist.view(np.int16)).cuda(), u, tgv.Params(iters=iters, schedule=tgv.SCHED_FUSED2))
    st = oracle.solve(hist, shape, scenes.default_bins(), iters, halo=1, u0=u0.astype(np.float64))
    assert np.abs(u.cpu().numpy() - st.u).max() <= 1e-5


def test_field_without_zero_level_has_no_crossings(ctx):
    import paper_2107_14790_amd as tgv
    say("no zero level")
    g = tgv.grid_c((0, 0, 0), 0.5, (33, 17, 9), 0)
    n = 33 * 17 * 9
    for u in (torch.ones(n, device="cuda"), -torch.ones(n, device="cuda"), torch.zeros(n, device="cuda")):
        assert ctx.extract_crossings(g, u).shape == (0, 4)


def test_large_depth_maps_histograms_bit_exact(ctx):
    """2048 x 2048 depth maps (12 pyramid levels; the precision workload's
    size) on a 48^3 block, with the voxels coarse enough to read from
    several levels: histograms bit for bit against the oracle."""
    import paper_2107_14790_amd as tgv
    say("2048^2 maps")
    sc = scenes.terrain_scene(n=48, n_side=2, W=2048, H=2048, f=3072.0, lattice=512, device="cuda")
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    opyr = oracle.pyramids(sc.depth)
    assert np.array_equal(pyr.cpu().numpy().reshape(-1).view(np.uint32), opyr.view(np.uint32))
    hist = ctx.build_histograms(pyr, W, H, sc.cams, tgv.grid_from(sc.grid)).cpu().numpy().view(np.uint16)
    ref, _ = oracle.histograms(sc, opyr)
    assert np.array_equal(hist, ref) and ref.sum() > 0
