"""Parity at the benchmark's full size and launch configuration.

The terrain block of the benchmark (256^3 voxels, 64 nadir 1024x1024 depth
maps) is too large for the oracle to solve whole, so it is checked where the
oracle can follow it exactly:

- histograms: bit-exact against the oracle on random voxels and on whole
  crops around surface points and block corners;
- solver: after N iterations a voxel depends only on voxels within Chebyshev
  distance 2 per iteration (the dual step reads x + e_i, the primal step
  x - e_i), so a crop that extends 2N + 2 voxels past a sample box on every
  side (clipped at the block's faces, where the masks are the block's own)
  gives the oracle exactly the values of the full solve in that box.  The
  oracle solves the crop from its own histograms; the GPU solves the whole
  block with the library defaults the benchmark uses;
- the full 1000-iteration solve of the benchmark, in its tiled launch
  configuration, is bit-identical to the per-voxel kernels (whose parity
  with the oracle the small-block tests establish);
- the rows that widen the path on the same block: histograms with
  terrestrial scans (vote 5) on random voxels, TV-L1 on crops, and the
  zero level of the solved block (count and the oracle's points of two
  rows)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu

N = 256
ITERS = 16


def say(*a):
    print("[fullsize]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def terrain():
    import paper_2107_14790_amd as tgv
    say("terrain scene 256^3, 64 cameras 1024x1024")
    sc = scenes.terrain_scene(n=N, n_side=8, W=1024, H=1024, f=1536.0, device="cuda")
    ctx = tgv.Context(0)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    g = tgv.grid_from(sc.grid)
    hist = ctx.build_histograms(pyr, W, H, tgv.cameras_from(sc.cams), g)
    torch.cuda.synchronize()
    say("oracle pyramids and histograms on 20000 random voxels")
    opyr = oracle.pyramids(sc.depth)
    rng = np.random.default_rng(2561)
    vox = rng.choice(N ** 3, size=20000, replace=False)
    ref, _ = oracle.histograms(sc, opyr, vox=vox)
    return dict(ctx=ctx, sc=sc, g=g, hist=hist, opyr=opyr, hist_np=hist.cpu().numpy().view(np.uint16),
                vox=vox, vox_hist=ref)


def crop_box(sample_lo, size, radius):
    lo = [max(0, s - radius) for s in sample_lo]
    hi = [min(N, s + size + radius) for s in sample_lo]
    return lo, hi


def crop_scene(sc, lo, hi):
    g = sc.grid
    o = np.asarray(g.origin, dtype=np.float64)
    origin = np.array([o[0] + lo[0] * g.h, o[1] + lo[1] * g.h, o[2] + lo[2] * g.h], dtype=np.float32)
    shape = tuple(h - l for l, h in zip(lo, hi))
    return scenes.Scene(sc.depth, sc.cams, scenes.Grid(origin, g.h, shape, 0)), shape


def crop_indices(lo, hi):
    z, y, x = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]), indexing="ij")
    return (x + N * y + N * N * z).ravel()


def test_histograms_on_random_voxels_bit_exact(terrain):
    ref = terrain["vox_hist"]
    assert np.array_equal(terrain["hist_np"][terrain["vox"]], ref)
    assert ref.sum() > 0


def surface_samples(vox, vox_hist, k, rng):
    """k of the oracle's random voxels with votes in the inner bins (near the surface)."""
    near = vox[np.nonzero(vox_hist[:, 1:6].sum(axis=1))[0]]
    idx = rng.choice(near, size=k, replace=False)
    return [(int(i % N), int((i // N) % N), int(i // (N * N))) for i in idx]


def test_solver_crops_match_oracle(terrain):
    """16 iterations on the whole block (library defaults, which run two
    iterations per pass at this size, as the benchmark does) against the
    oracle on crops around 4^3 sample boxes: at surface points, a block
    corner and an edge."""
    import paper_2107_14790_amd as tgv
    ctx, g = terrain["ctx"], terrain["g"]
    u = torch.zeros(N ** 3, device="cuda")
    ctx.solve(g, terrain["hist"], u, tgv.Params(iters=ITERS))
    torch.cuda.synchronize()
    u_gpu = u.cpu().numpy().reshape(N, N, N)
    rng = np.random.default_rng(2562)
    samples = surface_samples(terrain["vox"], terrain["vox_hist"], 3, rng)
    samples = [tuple(min(max(c - 2, 0), N - 4) for c in s) for s in samples] + [(0, 0, 0), (N - 4, N - 4, 100)]
    radius = 2 * ITERS + 2
    for s in samples:
        lo, hi = crop_box(s, 4, radius)
        csc, shape = crop_scene(terrain["sc"], lo, hi)
        say("crop", lo, hi)
        h_ref, _ = oracle.histograms(csc, terrain["opyr"])
        assert np.array_equal(terrain["hist_np"][crop_indices(lo, hi)], h_ref), "crop histograms"
        st = oracle.solve(h_ref, shape, scenes.default_bins(), ITERS)
        uc = st.u.reshape(shape[2], shape[1], shape[0])
        a = [s[i] - lo[i] for i in range(3)]
        ref = uc[a[2]:a[2] + 4, a[1]:a[1] + 4, a[0]:a[0] + 4]
        got = u_gpu[s[2]:s[2] + 4, s[1]:s[1] + 4, s[0]:s[0] + 4]
        assert np.abs(got - ref).max() <= 1e-4, s


def test_bench_solve_bit_identical_to_per_voxel_kernels(terrain):
    """The benchmark's 1000 iterations in its launch configuration (two
    iterations per pass) and with one tiled pass per iteration, against the
    same solve with the per-voxel dual and primal kernels."""
    import paper_2107_14790_amd as tgv
    ctx, g = terrain["ctx"], terrain["g"]
    out = []
    for sched in (tgv.SCHED_FUSED2, tgv.SCHED_FUSED, tgv.SCHED_SPLIT):
        say("1000 iterations, schedule", sched)
        u = torch.zeros(N ** 3, device="cuda")
        st = ctx.solve(g, terrain["hist"], u, tgv.Params(iters=1000, schedule=sched), stats=True)
        torch.cuda.synchronize()
        assert st["nonfinite"] == 0
        out.append(u.cpu().numpy())
    assert np.array_equal(out[0].view(np.uint32), out[2].view(np.uint32))
    assert np.array_equal(out[1].view(np.uint32), out[2].view(np.uint32))


def test_scan_histograms_on_random_voxels_bit_exact(terrain):
    """Four terrestrial 360-degree scans (equirectangular, 4096 x 2048,
    vote 5) fused with the 64 stereo maps of 1024^2 in one call: histograms
    of the whole block on random voxels against the oracle."""
    import paper_2107_14790_amd as tgv
    ctx, sc = terrain["ctx"], terrain["sc"]
    say("terrain scans: 4 scanners 4096 x 2048")
    sd, scams = scenes.terrain_scans360(n=N, device="cuda")
    cams = scenes.concat_cameras(sc.cams, scams)
    pyr, offs = ctx.build_pyramids_mixed([torch.from_numpy(sc.depth).cuda(), torch.from_numpy(sd).cuda()])
    hist = ctx.build_histograms_ex(pyr, offs, cams, terrain["g"])
    got = hist.cpu().numpy().view(np.uint16)
    rng = np.random.default_rng(2563)
    vox = rng.choice(N ** 3, size=20000, replace=False)
    say("oracle on 20000 random voxels x", len(cams), "maps")
    opyr = np.concatenate([terrain["opyr"], oracle.pyramids(sd)])
    ref, _ = oracle.histograms(scenes.Scene(None, cams, sc.grid), opyr, vox=vox)
    assert np.array_equal(got[vox], ref)
    # the scans add votes of weight 5 near the ground around the scanners
    assert (got[vox].astype(np.int64) - terrain["hist_np"][vox]).max() >= 5


def test_tvl1_crops_match_oracle(terrain):
    """The TV-L1 model (Eq. 1) on the whole block, 16 iterations with the
    library defaults, against the oracle on crops (the same locality
    argument as for TGV)."""
    import paper_2107_14790_amd as tgv
    ctx, g = terrain["ctx"], terrain["g"]
    u = torch.zeros(N ** 3, device="cuda")
    ctx.solve(g, terrain["hist"], u, tgv.Params(iters=ITERS, flags=tgv.FLAG_TVL1))
    torch.cuda.synchronize()
    u_gpu = u.cpu().numpy().reshape(N, N, N)
    rng = np.random.default_rng(2564)
    samples = surface_samples(terrain["vox"], terrain["vox_hist"], 2, rng)
    samples = [tuple(min(max(c - 2, 0), N - 4) for c in s) for s in samples] + [(N - 4, 0, 120)]
    radius = 2 * ITERS + 2
    for s in samples:
        lo, hi = crop_box(s, 4, radius)
        csc, shape = crop_scene(terrain["sc"], lo, hi)
        say("tvl1 crop", lo, hi)
        h_ref, _ = oracle.histograms(csc, terrain["opyr"])
        assert np.array_equal(terrain["hist_np"][crop_indices(lo, hi)], h_ref), "crop histograms"
        st = oracle.solve(h_ref, shape, scenes.default_bins(), ITERS, tvl1=True)
        uc = st.u.reshape(shape[2], shape[1], shape[0])
        a = [s[i] - lo[i] for i in range(3)]
        ref = uc[a[2]:a[2] + 4, a[1]:a[1] + 4, a[0]:a[0] + 4]
        got = u_gpu[s[2]:s[2] + 4, s[1]:s[1] + 4, s[0]:s[0] + 4]
        assert np.abs(got - ref).max() <= 1e-4, s


def test_zero_level_of_the_solved_block(terrain):
    """Crossings of the whole solved block (200 iterations): their number is
    the number of sign-changing grid edges counted here independently, and
    the oracle's points of the two bottom rows (y = 0, 1; the same origin,
    so the same float32 arithmetic) are all among them, bit for bit."""
    import paper_2107_14790_amd as tgv
    ctx, g, sc = terrain["ctx"], terrain["g"], terrain["sc"]
    u = torch.zeros(N ** 3, device="cuda")
    ctx.solve(g, terrain["hist"], u, tgv.Params(iters=200))
    pts = ctx.extract_crossings(g, u).cpu().numpy()
    U = u.cpu().numpy().reshape(N, N, N)
    pos = U > 0
    edges = sum(int((pos.take(range(1, N), axis=ax) != pos.take(range(0, N - 1), axis=ax)).sum()) for ax in range(3))
    say("zero level:", len(pts), "points, sign-changing edges", edges)
    assert len(pts) == edges and edges > N * N
    crop = np.ascontiguousarray(U[:, 0:2, :])
    ref = oracle.crossings(crop.ravel(), (N, 2, N), sc.grid.origin, sc.grid.h)
    assert len(ref) > 0
    got = {r.tobytes() for r in pts.view(np.uint32)}
    assert all(r.tobytes() in got for r in ref.view(np.uint32))


# ---------------------------------------------------------------------------
# The whole block against the oracle at the benchmark's iteration count.
# Both sides advance together in chunks of CHUNK iterations (the GPU on a
# resumable state with the library's default schedule, two iterations per
# pass here, as the benchmark runs; the oracle on its own float64 state with
# its per-voxel loops on the host's cores, bit-identical to its serial run);
# each chunk is compared element by element over all 256^3 voxels.  A GPU
# solve resumed in chunks is bit-identical to one uninterrupted solve, which
# the last test checks against the benchmark's own call.
# ---------------------------------------------------------------------------
CHUNK = 200
FULL_ITERS = 1000


@pytest.fixture(scope="module")
def whole_block(terrain):
    import os
    import paper_2107_14790_amd as tgv
    sc = terrain["sc"]
    k = max(1, min(16, os.cpu_count() or 1))
    say(f"oracle histograms of all {N}^3 voxels x 64 maps on {k} threads")
    with oracle.threads(k):
        h_ref, _ = oracle.histograms(sc, terrain["opyr"])
    assert np.array_equal(terrain["hist_np"], h_ref), "whole-block histograms differ from the oracle"
    ctx, g = terrain["ctx"], terrain["g"]
    st = tgv.State(ctx, g)
    st.reset(torch.zeros(N ** 3, device="cuda"))
    return dict(k=k, h_ref=h_ref, gpu=st, ora=None, done=[0])


def advance_to(wb, terrain, iters):
    import paper_2107_14790_amd as tgv
    ctx, g = terrain["ctx"], terrain["g"]
    while wb["done"][0] < iters:
        step = min(CHUNK, iters - wb["done"][0])
        ctx.solve(g, terrain["hist"], None, tgv.Params(iters=step), state=wb["gpu"])
        with oracle.threads(wb["k"]):
            wb["ora"] = oracle.solve(wb["h_ref"], (N, N, N), scenes.default_bins(), step, state=wb["ora"])
        wb["done"][0] += step
        say(f"both sides at {wb['done'][0]} iterations")


@pytest.mark.parametrize("iters", list(range(CHUNK, FULL_ITERS + 1, CHUNK)))
def test_whole_block_matches_oracle(whole_block, terrain, iters):
    """max |u_gpu - u_oracle| <= 1e-4 over every voxel of the 256^3 block
    after 200, 400, ..., 1000 iterations."""
    advance_to(whole_block, terrain, iters)
    got = whole_block["gpu"].export()["u"].cpu().numpy().astype(np.float64)
    err = np.abs(got - whole_block["ora"].u)
    say(f"{iters} iterations: max |u - u_oracle| = {err.max():.3g}, mean {err.mean():.3g}")
    assert np.isfinite(got).all()
    assert err.max() <= 1e-4


def test_whole_block_benchmark_call_equals_chunked_solve(whole_block, terrain):
    """The benchmark's call (a fresh 1000-iteration solve with the library's
    defaults) gives the chunked solve's u bit for bit, so the oracle
    comparison above holds for it."""
    import paper_2107_14790_amd as tgv
    advance_to(whole_block, terrain, FULL_ITERS)
    ctx, g = terrain["ctx"], terrain["g"]
    u = torch.zeros(N ** 3, device="cuda")
    ctx.solve(g, terrain["hist"], u, tgv.Params(iters=FULL_ITERS))
    chunked = whole_block["gpu"].export()["u"]
    assert torch.equal(u, chunked)
