"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Histograms and pyramids bit-exact; u within 1e-4
max-abs of the float64 oracle; energies within float64 reduction error."""
import sys

import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu

TAU = float(np.float32(1.0 / np.sqrt(12.0)))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    return tgv.Context(0)


def gpu_hist(ctx, sc, rule=0, num_bins=7):
    import paper_2107_14790_amd as tgv
    d = torch.from_numpy(sc.depth).cuda()
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(d)
    hist = ctx.build_histograms(pyr, W, H, sc.cams, sc.grid, tgv.Bins(num_bins=num_bins, rule=rule))
    torch.cuda.synchronize()
    return pyr.cpu().numpy(), hist.cpu().numpy().view(np.uint16)


# ---------------------------------------------------------------------------
# pyramids and histograms: bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("W,H", [(128, 128), (100, 75), (7, 3), (1, 1), (513, 257)])
def test_pyramids_bit_exact(ctx, W, H):
    say("pyramids", W, H)
    rng = np.random.default_rng(W * 1000 + H)
    d = rng.uniform(0.5, 3.0, size=(3, H, W)).astype(np.float32)
    d[rng.random(d.shape) < 0.2] = 0.0
    d[rng.random(d.shape) < 0.05] = np.nan
    d[rng.random(d.shape) < 0.05] = -1.0
    d[rng.random(d.shape) < 0.02] = np.inf
    pyr = ctx.build_pyramids(torch.from_numpy(d).cuda()).cpu().numpy()
    for c in range(3):
        ref = oracle.pyramid(d[c])
        assert np.array_equal(pyr[c].view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("rule", [0, 1])
def test_sphere_histograms_bit_exact(ctx, rule):
    say("sphere32 histograms rule", rule)
    sc = scenes.sphere_scene()
    pyr, hist = gpu_hist(ctx, sc, rule=rule)
    ref_pyr = oracle.pyramids(sc.depth)
    assert np.array_equal(pyr.reshape(-1).view(np.uint32), ref_pyr.view(np.uint32))
    ref, _ = oracle.histograms(sc, ref_pyr, rule=rule)
    assert np.array_equal(hist, ref)
    assert hist.sum() > 0


@pytest.mark.parametrize("num_bins", [1, 2, 5, 8])
def test_histograms_other_bin_counts(ctx, num_bins):
    say("sphere16 histograms bins", num_bins)
    sc = scenes.sphere_scene(n=16)
    for rule in (0, 1):
        _, hist = gpu_hist(ctx, sc, rule=rule, num_bins=num_bins)
        ref, _ = oracle.histograms(sc, rule=rule, num_bins=num_bins)
        assert np.array_equal(hist, ref)


def test_ragged_terrain_histograms_bit_exact(ctx):
    # several 64x4 tiles plus ragged tails in x and y, mip levels > 0
    say("terrain ragged histograms")
    sc = scenes.terrain_scene(n=40, n_side=3, W=160, H=144, f=200.0, lattice=256)
    sc.grid.n = (70, 37, 23)
    pyr, hist = gpu_hist(ctx, sc)
    ref, _ = oracle.histograms(sc)
    assert np.array_equal(hist, ref)


def test_votes_weights_and_plane(ctx):
    say("plane histograms with vote weights")
    sc = scenes.plane_scene(n=(5, 4, 28), z_plane_index=12, n_cams=4)
    sc.cams.vote[:] = [1, 5, 3, 5]
    _, hist = gpu_hist(ctx, sc)
    ref, _ = oracle.histograms(sc)
    assert np.array_equal(hist, ref)


def test_histogram_overflow_and_bad_args(ctx):
    import paper_2107_14790_amd as tgv
    say("histogram overflow error")
    sc = scenes.plane_scene(n=(2, 2, 3), z_plane_index=1, n_cams=2)
    sc.cams.vote[:] = [40000, 40000]
    d = torch.from_numpy(sc.depth).cuda()
    pyr = ctx.build_pyramids(d)
    with pytest.raises(tgv.TgvError) as e:
        ctx.build_histograms(pyr, 64, 64, sc.cams, sc.grid)
    assert e.value.status == tgv.TGV_E_OVERFLOW
    with pytest.raises(tgv.TgvError) as e:
        ctx.build_histograms(pyr, 64, 64, sc.cams, sc.grid, tgv.Bins(num_bins=9))
    assert e.value.status == tgv.TGV_E_INVAL
    with pytest.raises(tgv.TgvError) as e:
        ctx.build_histograms(pyr, 32, 64, sc.cams, sc.grid)  # camera size mismatch
    assert e.value.status == tgv.TGV_E_INVAL


# ---------------------------------------------------------------------------
# solver
# ---------------------------------------------------------------------------
def solve_gpu(ctx, hist_np, shape, iters, halo=0, u0=None, storage=0, schedule=0, alpha0=2.0, alpha1=1.0,
              lam=1.0, tau=TAU, stats=False):
    import paper_2107_14790_amd as tgv
    nx, ny, nz = shape
    n = nx * ny * nz
    g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
    hist = torch.from_numpy(hist_np.view(np.int16).reshape(n, 8)).cuda()
    u = torch.zeros(n, device="cuda") if u0 is None else torch.from_numpy(np.asarray(u0, np.float32)).cuda()
    p = tgv.Params(alpha0=alpha0, alpha1=alpha1, lam=lam, tau=tau, sigma=tau, iters=iters, storage=storage,
                   schedule=schedule)
    st = ctx.solve(g, hist, u, p, stats=stats)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64), st


def test_sphere32_u_matches_oracle(ctx):
    say("sphere32 solve 300 iterations")
    sc = scenes.sphere_scene()
    ref_h, _ = oracle.histograms(sc)
    _, hist = gpu_hist(ctx, sc)
    assert np.array_equal(hist, ref_h)
    u_gpu, stats = solve_gpu(ctx, hist, (32, 32, 32), 300, stats=True)
    st = oracle.solve(ref_h, (32, 32, 32), scenes.default_bins(), 300)
    err = np.abs(u_gpu - st.u).max()
    say("sphere32 max|u_gpu - u_oracle| =", err)
    assert err <= 1e-4
    P, D, g = oracle.gap(ref_h, (32, 32, 32), scenes.default_bins(), st)
    assert abs(stats["primal"] - P) <= 1e-4 * P
    assert stats["nonfinite"] == 0 and stats["iters_done"] == 300


@pytest.mark.parametrize("shape,halo,iters", [((37, 29, 23), 2, 120), ((70, 9, 5), 0, 200), ((1, 1, 1), 0, 10),
                                              ((17, 1, 1), 0, 150), ((1, 13, 6), 0, 90), ((64, 8, 8), 3, 60)])
def test_ragged_blocks_match_oracle(ctx, shape, halo, iters):
    say("ragged solve", shape, halo, iters)
    rng = np.random.default_rng(sum(shape) + halo)
    n = int(np.prod(shape))
    hist = np.zeros((n, 8), dtype=np.uint16)
    tot = rng.integers(0, 12, size=n)
    for x in range(n):
        if tot[x]:
            hist[x, :7] = np.bincount(rng.integers(0, 7, size=tot[x]), minlength=7)
    u0 = np.where(rng.random(n) < 0.5, rng.uniform(-1, 1, n), 0.0).astype(np.float32)
    u_gpu, _ = solve_gpu(ctx, hist, shape, iters, halo=halo, u0=u0)
    st = oracle.solve(hist, shape, scenes.default_bins(), iters, halo=halo, u0=u0.astype(np.float64))
    assert np.abs(u_gpu - st.u).max() <= 1e-4
    if halo:
        nx, ny, nz = shape
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        fr = ((x < halo) | (y < halo) | (z < halo) | (x >= nx - halo) | (y >= ny - halo) | (z >= nz - halo)).ravel()
        assert np.array_equal(u_gpu[fr], u0[fr].astype(np.float64))


def test_fused_and_split_schedules_bit_identical(ctx):
    say("fused vs split")
    sc = scenes.sphere_scene(n=24)
    _, hist = gpu_hist(ctx, sc)
    a, _ = solve_gpu(ctx, hist, (24, 24, 24), 57, schedule=0)
    b, _ = solve_gpu(ctx, hist, (24, 24, 24), 57, schedule=1)
    assert np.array_equal(a, b)


def test_resume_is_bitwise_and_export_import_roundtrip(ctx):
    import paper_2107_14790_amd as tgv
    say("resume / export / import")
    sc = scenes.sphere_scene(n=20)
    _, hist_np = gpu_hist(ctx, sc)
    g = tgv.grid_from(sc.grid)
    n = 20 ** 3
    hist = torch.from_numpy(hist_np.view(np.int16)).cuda()
    u0 = torch.zeros(n, device="cuda")
    full = tgv.State(ctx, g)
    full.reset(u0)
    ctx.solve(g, hist, None, tgv.Params(iters=90), state=full)
    part = tgv.State(ctx, g)
    part.reset(u0)
    ctx.solve(g, hist, None, tgv.Params(iters=40), state=part)
    f = part.export()
    other = tgv.State(ctx, g)
    other.import_(f, iters_done=40)
    ctx.solve(g, hist, None, tgv.Params(iters=50), state=other)
    ctx.solve(g, hist, None, tgv.Params(iters=50), state=part)
    a, b, c = full.export(), part.export(), other.export()
    for k in a:
        assert torch.equal(a[k], b[k]), k
        assert torch.equal(a[k], c[k]), k


def test_state_fields_match_oracle(ctx):
    import paper_2107_14790_amd as tgv
    say("state fields vs oracle")
    sc = scenes.sphere_scene(n=16)
    ref_h, _ = oracle.histograms(sc)
    g = tgv.grid_from(sc.grid)
    hist = torch.from_numpy(ref_h.view(np.int16)).cuda()
    st = tgv.State(ctx, g)
    st.reset(torch.zeros(16 ** 3, device="cuda"))
    ctx.solve(g, hist, None, tgv.Params(iters=100), state=st)
    f = {k: v.cpu().numpy().astype(np.float64) for k, v in st.export().items()}
    ref = oracle.solve(ref_h, (16, 16, 16), scenes.default_bins(), 100)
    for k in ("u", "v", "p", "q"):
        assert np.abs(f[k] - getattr(ref, k)).max() <= 1e-4, k
    # ubar = 2 u - u_prev
    assert np.abs((2 * f["u"] - f["u_prev"]) - ref.ubar).max() <= 2e-4


def test_energy_reduction_matches_oracle_on_same_fields(ctx):
    import paper_2107_14790_amd as tgv
    say("energy parity")
    sc = scenes.sphere_scene(n=24)
    ref_h, _ = oracle.histograms(sc)
    g = tgv.grid_c(sc.grid.origin, sc.grid.h, (24, 24, 24), 2)
    hist = torch.from_numpy(ref_h.view(np.int16)).cuda()
    st = tgv.State(ctx, g)
    st.reset(torch.zeros(24 ** 3, device="cuda"))
    ctx.solve(g, hist, None, tgv.Params(iters=80), state=st)
    s = ctx.energy(st, hist)
    f = {k: v.cpu().numpy().astype(np.float64) for k, v in st.export().items()}
    c = scenes.default_bins()
    P, parts = oracle.primal_energy(ref_h, (24, 24, 24), c, f["u"], f["v"], halo=2)
    D = oracle.dual_energy(ref_h, (24, 24, 24), c, f["u"], f["p"], f["q"], halo=2)
    assert abs(s["primal"] - P) <= 1e-9 * abs(P)
    np.testing.assert_allclose(s["parts"], parts, rtol=1e-9)
    assert abs(s["dual"] - D) <= 1e-9 * max(1.0, abs(D))
    assert s["nonfinite"] == 0


def test_gap_decreases_like_the_oracle(ctx):
    # the relative gap closes at the sublinear rate of the primal-dual method;
    # the GPU's float64 reduction of its float32 iterates tracks the oracle
    say("gap decreases")
    rng = np.random.default_rng(3)
    shape = (8, 8, 8)
    n = 512
    hist = np.zeros((n, 8), dtype=np.uint16)
    for x in range(n):
        hist[x, :7] = np.bincount(rng.integers(0, 7, size=2 * rng.integers(0, 5) + 1), minlength=7)
    gaps, ref = [], []
    st = None
    prev = 0
    for it in (100, 1000, 10000):
        _, s = solve_gpu(ctx, hist, shape, it, stats=True)
        gaps.append(s["gap_rel"])
        st = oracle.solve(hist, shape, scenes.default_bins(), it - prev, state=st)
        prev = it
        ref.append(oracle.gap(hist, shape, scenes.default_bins(), st)[2])
    assert gaps[0] > gaps[1] > gaps[2]
    for a, b in zip(gaps, ref):
        assert abs(a - b) <= 1e-2 * b + 1e-6, (gaps, ref)


def test_zero_iterations_and_alpha_zero_median(ctx):
    say("iters=0 and alpha=0")
    rng = np.random.default_rng(9)
    shape = (9, 7, 5)
    n = 315
    hist = np.zeros((n, 8), dtype=np.uint16)
    for x in range(n):
        hist[x, :7] = np.bincount(rng.integers(0, 7, size=2 * rng.integers(0, 4) + 1), minlength=7)
    u0 = rng.uniform(-1, 1, n).astype(np.float32)
    u, _ = solve_gpu(ctx, hist, shape, 0, u0=u0)
    assert np.array_equal(u, u0.astype(np.float64))
    u, _ = solve_gpu(ctx, hist, shape, 100, alpha0=0.0, alpha1=0.0)
    c = scenes.default_bins()[:7].astype(np.float64)
    med = np.array([oracle.weighted_median_interval(hist[x, :7].astype(int), c)[0] for x in range(n)])
    assert np.array_equal(u, np.float32(med).astype(np.float64))


# unit roundoff of the storage format of v, p, q (FP16: 11-bit significand,
# BF16: 8-bit)
UNIT_ROUNDOFF = {1: 2.0 ** -11, 2: 2.0 ** -8}


def zero_crossings(u, ref):
    """Crossing positions t = u_a / (u_a - u_b) on the grid edges where both
    fields change sign (in voxels): |t - t_ref| per such edge."""
    a, b = u.reshape(32, 32, 32), ref.reshape(32, 32, 32)
    out = []
    for ax in range(3):
        a0, a1 = np.moveaxis(a, ax, 0)[:-1], np.moveaxis(a, ax, 0)[1:]
        b0, b1 = np.moveaxis(b, ax, 0)[:-1], np.moveaxis(b, ax, 0)[1:]
        both = ((a0 > 0) != (a1 > 0)) & ((b0 > 0) != (b1 > 0))
        out.append(np.abs(a0[both] / (a0[both] - a1[both]) - b0[both] / (b0[both] - b1[both])))
    return np.concatenate(out)


def test_half_storage_close_to_oracle(ctx):
    """16-bit storage of v, p, q against the float64 oracle after 300
    iterations on the sphere block.  The deviation is a storage rounding
    effect: in units of each format's unit roundoff u_s (FP16 2^-11, BF16
    2^-8) it stays within the stated bounds, max |u - u_64| <= 128 u_s,
    mean |u - u_64| <= u_s and a mean zero-crossing shift <= 8 u_s voxel,
    and BF16's mean deviation is 2 to 32 times FP16's, as the ratio of their
    unit roundoffs (8) predicts for rounding, not for a defect of one path."""
    sc = scenes.sphere_scene()
    ref_h, _ = oracle.histograms(sc)
    st = oracle.solve(ref_h, (32, 32, 32), scenes.default_bins(), 300)
    mean = {}
    for storage in (1, 2):
        say("half storage", storage)
        u16, s = solve_gpu(ctx, ref_h, (32, 32, 32), 300, storage=storage, stats=True)
        us = UNIT_ROUNDOFF[storage]
        d = np.abs(u16 - st.u)
        zc = zero_crossings(u16.astype(np.float64), st.u)
        say("storage", storage, "max", d.max() / us, "mean", d.mean() / us, "zc mean", zc.mean() / us, "u_s")
        assert s["nonfinite"] == 0 and zc.size > 1000
        assert d.max() <= 128 * us
        assert d.mean() <= us
        assert zc.mean() <= 8 * us
        mean[storage] = d.mean()
    assert 2.0 <= mean[2] / mean[1] <= 32.0


# ---------------------------------------------------------------------------
# the tiled fused kernel reproduces the reference kernels bit for bit
# ---------------------------------------------------------------------------
def _full_state(ctx, hist_np, shape, iters, halo, u0, params):
    import paper_2107_14790_amd as tgv
    n = int(np.prod(shape))
    g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
    hist = torch.from_numpy(hist_np.view(np.int16).reshape(n, 8)).cuda()
    st = tgv.State(ctx, g, params.storage)
    st.reset(torch.from_numpy(u0).cuda())
    ctx.solve(g, hist, None, params, state=st)
    out = {k: v.cpu().numpy() for k, v in st.export().items()}
    st.close()
    return out


@pytest.mark.parametrize("shape,halo", [((70, 37, 23), 2), ((130, 20, 67), 0), ((64, 8, 32), 1), ((5, 3, 40), 0),
                                        ((200, 1, 3), 0), ((37, 29, 23), 2)])
@pytest.mark.parametrize("storage", [0, 1, 2])
def test_tiled_kernel_bitwise_equals_split(ctx, shape, halo, storage):
    import paper_2107_14790_amd as tgv
    say("tiled vs split", shape, halo, storage)
    rng = np.random.default_rng(sum(shape) * 7 + storage)
    n = int(np.prod(shape))
    hist = np.zeros((n, 8), dtype=np.uint16)
    tot = rng.integers(0, 10, size=n)
    b = rng.integers(0, 7, size=int(tot.sum()))
    np.add.at(hist, (np.repeat(np.arange(n), tot), b), 1)
    u0 = np.where(rng.random(n) < 0.5, rng.uniform(-1, 1, n), 0.0).astype(np.float32)
    ref = _full_state(ctx, hist, shape, 23, halo, u0, tgv.Params(iters=23, storage=storage,
                                                                schedule=tgv.SCHED_SPLIT))
    for ty, cz in [(8, 32), (4, 5), (12, 1), (8, 7)]:
        got = _full_state(ctx, hist, shape, 23, halo, u0,
                          tgv.Params(iters=23, storage=storage, tile_y=ty, tile_z=cz))
        for k in ref:
            assert np.array_equal(ref[k].view(np.uint32), got[k].view(np.uint32)), (k, ty, cz)


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_streamed_store_path_bitwise_equals_split(ctx, storage):
    """A block whose iteration moves more than 256 MiB (160^3: 491 MB in
    float32, 295 MB in 16-bit storage) takes the non-temporal store path and,
    in float32, the 64 x 8 default tile; bit-identical to the per-voxel
    kernels all the same."""
    import paper_2107_14790_amd as tgv
    shape = (160, 160, 160)
    say("streamed stores", shape, storage)
    rng = np.random.default_rng(160 + storage)
    n = int(np.prod(shape))
    hist = np.zeros((n, 8), dtype=np.uint16)
    hist[:, :7] = rng.integers(0, 3, size=(n, 7), dtype=np.uint16) * (rng.random((n, 1)) < 0.4)
    u0 = np.where(rng.random(n) < 0.5, rng.uniform(-1, 1, n), 0.0).astype(np.float32)
    ref = _full_state(ctx, hist, shape, 9, 0, u0, tgv.Params(iters=9, storage=storage, schedule=tgv.SCHED_SPLIT))
    for ty, cz in [(0, 0), (4, 32)]:
        got = _full_state(ctx, hist, shape, 9, 0, u0, tgv.Params(iters=9, storage=storage, tile_y=ty, tile_z=cz,
                                                                schedule=tgv.SCHED_FUSED))
        for k in ref:
            assert np.array_equal(ref[k].view(np.uint32), got[k].view(np.uint32)), (k, ty, cz)


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_state_reset_clears_every_element_of_odd_sized_blocks(ctx, storage):
    """A state whose memory held NaN: after a reset v, p and q are exactly 0
    and u is u0, including the last element of 16-bit arrays of an odd voxel
    count (3 n or 6 n half words)."""
    import paper_2107_14790_amd as tgv
    for shape in ((37, 29, 23), (1, 1, 1), (3, 5, 7)):
        n = int(np.prod(shape))
        g = tgv.grid_c((0, 0, 0), 1.0, shape, 0)
        mem = torch.full((tgv.state_bytes(g, storage) // 4,), float("nan"), device="cuda")
        st = tgv.State(ctx, g, storage, memory=mem)
        u0 = torch.linspace(-1, 1, n, device="cuda")
        st.reset(u0)
        f = st.export()
        torch.cuda.synchronize()
        for k in ("v", "v_prev", "p", "q"):
            assert torch.count_nonzero(f[k]).item() == 0, (shape, k)
        assert torch.equal(f["u"], u0) and torch.equal(f["u_prev"], u0)
        st.close()


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_fused_reference_schedule_bitwise_equals_split(ctx, storage):
    """The per-voxel fused kernel (schedule FUSED_REF, also the path of blocks
    too large for the tiled kernel's 32-bit offsets) against the split one."""
    import paper_2107_14790_amd as tgv
    for shape, halo in (((37, 29, 23), 2), ((130, 9, 5), 0), ((1, 1, 1), 0)):
        say("fused_ref vs split", shape, halo, storage)
        rng = np.random.default_rng(sum(shape) + 31 * storage)
        n = int(np.prod(shape))
        hist = np.zeros((n, 8), dtype=np.uint16)
        hist[:, :7] = rng.integers(0, 4, size=(n, 7), dtype=np.uint16) * (rng.random((n, 1)) < 0.5)
        u0 = np.where(rng.random(n) < 0.5, rng.uniform(-1, 1, n), 0.0).astype(np.float32)
        ref = _full_state(ctx, hist, shape, 17, halo, u0, tgv.Params(iters=17, storage=storage,
                                                                    schedule=tgv.SCHED_SPLIT))
        got = _full_state(ctx, hist, shape, 17, halo, u0, tgv.Params(iters=17, storage=storage,
                                                                    schedule=tgv.SCHED_FUSED_REF))
        for k in ref:
            assert np.array_equal(ref[k].view(np.uint32), got[k].view(np.uint32)), k


def test_block_beyond_tiled_offsets_falls_back_correctly(ctx):
    """448^3 voxels: 24 n >= 2^31, so the fused passes run the per-voxel
    fused kernel.  Bitwise equal to the split schedule, and equal to the
    oracle on a corner crop (4 iterations reach at most 2 voxels each)."""
    import paper_2107_14790_amd as tgv
    shape = (448, 448, 448)
    n = int(np.prod(shape))
    assert 24 * n >= 2 ** 31
    say("fallback block", shape)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(448)
    hist = torch.zeros((n, 8), dtype=torch.int16, device="cuda")
    hist[:, :7] = torch.randint(0, 3, (n, 7), device="cuda", dtype=torch.int16, generator=gen)
    hist[torch.rand(n, device="cuda", generator=gen) < 0.6] = 0
    g = tgv.grid_c((0, 0, 0), 1.0, shape, 0)
    out = []
    for sched in (tgv.SCHED_FUSED, tgv.SCHED_SPLIT):
        u = torch.zeros(n, device="cuda")
        ctx.solve(g, hist, u, tgv.Params(iters=4, schedule=sched))
        torch.cuda.synchronize()
        out.append(u.cpu().numpy())
    assert np.array_equal(out[0].view(np.uint32), out[1].view(np.uint32))
    c = 14  # corner crop: sample 4^3 at the origin, 2 * 4 + 2 voxels of context
    hc = hist.view(shape[2], shape[1], shape[0], 8)[:c, :c, :c].contiguous().cpu().numpy()
    st = oracle.solve(hc.reshape(-1, 8).view(np.uint16), (c, c, c), scenes.default_bins(), 4)
    ref = st.u.reshape(c, c, c)[:4, :4, :4]
    got = out[0].reshape(shape[2], shape[1], shape[0])[:4, :4, :4]
    assert np.abs(got - ref).max() <= 1e-4
    del hist


# ---------------------------------------------------------------------------
# zero-level points
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(37, 29, 23), (64, 8, 9), (1, 1, 1), (300, 3, 2), (70, 64, 60)])
def test_crossings_bit_exact(ctx, shape):
    say("crossings", shape)
    rng = np.random.default_rng(sum(shape))
    n = int(np.prod(shape))
    u = rng.uniform(-1, 1, n).astype(np.float32)
    u[rng.random(n) < 0.1] = 0.0
    origin = np.array([-0.3, 0.1, 2.0], dtype=np.float32)
    h = 0.0625
    import paper_2107_14790_amd as tgv
    g = tgv.grid_c(origin, h, shape, 0)
    pts = ctx.extract_crossings(g, torch.from_numpy(u).cuda()).cpu().numpy()
    ref = oracle.crossings(u, shape, origin, h)
    assert pts.shape == ref.shape
    assert np.array_equal(pts.view(np.uint32), ref.view(np.uint32))


def test_crossings_into_preallocated_output(ctx):
    import paper_2107_14790_amd as tgv
    say("crossings into a preallocated output")
    rng = np.random.default_rng(5)
    shape = (40, 33, 17)
    u = torch.from_numpy(rng.uniform(-1, 1, int(np.prod(shape))).astype(np.float32)).cuda()
    g = tgv.grid_c((0.5, -1.0, 0.25), 0.125, shape, 0)
    ref = ctx.extract_crossings(g, u)
    out = torch.full((ref.shape[0] + 7, 4), -1.0, device="cuda")
    got = ctx.extract_crossings(g, u, out=out)
    assert torch.equal(got, ref)
    assert torch.equal(out[ref.shape[0]:], torch.full((7, 4), -1.0, device="cuda"))  # rows past the count untouched
    with pytest.raises(ValueError):
        ctx.extract_crossings(g, u, out=torch.empty((ref.shape[0] - 1, 4), device="cuda"))


def test_crossings_of_solved_sphere(ctx):
    say("sphere crossings")
    sc = scenes.sphere_scene()
    ref_h, _ = oracle.histograms(sc)
    u, _ = solve_gpu(ctx, ref_h, (32, 32, 32), 300)
    u32 = u.astype(np.float32)
    import paper_2107_14790_amd as tgv
    g = tgv.grid_from(sc.grid)
    pts = ctx.extract_crossings(g, torch.from_numpy(u32).cuda()).cpu().numpy()
    ref = oracle.crossings(u32, (32, 32, 32), sc.grid.origin, sc.grid.h)
    assert np.array_equal(pts.view(np.uint32), ref.view(np.uint32))
    # the ring cameras see the sphere near their plane; above and below it
    # the data term is empty and u hovers around 0, so only that band is
    # checked against the unit sphere
    band = np.abs(pts[:, 2]) < 0.5
    r = np.linalg.norm(pts[band, :3], axis=1)
    assert band.sum() > 500 and np.median(np.abs(r - 1.0)) < 0.03 and np.percentile(np.abs(r - 1.0), 90) < 0.06


# ---------------------------------------------------------------------------
# coarse-to-fine
# ---------------------------------------------------------------------------
def test_prolongate_matches_oracle(ctx):
    import paper_2107_14790_amd as tgv
    say("prolongate")
    rng = np.random.default_rng(4)
    uc = rng.normal(size=5 * 4 * 3).astype(np.float32)
    gc = tgv.grid_c((0, 0, 0), 2.0, (5, 4, 3))
    gf = tgv.grid_c((0, 0, 0), 1.0, (9, 8, 6))
    out = ctx.prolongate(gc, torch.from_numpy(uc).cuda(), gf).cpu().numpy()
    assert np.array_equal(out, oracle.prolongate(uc, (5, 4, 3), (9, 8, 6)).astype(np.float32))
    with pytest.raises(tgv.TgvError):
        ctx.prolongate(gc, torch.from_numpy(uc).cuda(), tgv.grid_c((0, 0, 0), 1.0, (12, 8, 6)))


@pytest.mark.parametrize("levels", [2, 3])
def test_coarse_to_fine_matches_oracle(ctx, levels):
    import paper_2107_14790_amd as tgv
    say("coarse to fine", levels)
    sc = scenes.sphere_scene(n=32)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    u = ctx.solve_coarse_to_fine(pyr, W, H, sc.cams, sc.grid, levels, tgv.Params(iters=100)).cpu().numpy()
    ref = oracle.coarse_to_fine(sc, levels, 100)
    assert np.abs(u.astype(np.float64) - ref).max() <= 1e-4


# ---------------------------------------------------------------------------
# TV-L1 model (Eq. 1)
# ---------------------------------------------------------------------------
def test_tvl1_matches_oracle(ctx):
    import paper_2107_14790_amd as tgv
    say("tv-l1")
    sc = scenes.sphere_scene()
    ref_h, _ = oracle.histograms(sc)
    g = tgv.grid_from(sc.grid)
    hist = torch.from_numpy(ref_h.view(np.int16)).cuda()
    st = tgv.State(ctx, g)
    st.reset(torch.zeros(32 ** 3, device="cuda"))
    stats = ctx.solve(g, hist, None, tgv.Params(iters=300, flags=tgv.FLAG_TVL1), state=st, stats=True)
    f = {k: v.cpu().numpy().astype(np.float64) for k, v in st.export().items()}
    ref = oracle.solve(ref_h, (32, 32, 32), scenes.default_bins(), 300, tvl1=True)
    assert np.abs(f["u"] - ref.u).max() <= 1e-4
    assert not f["v"].any() and not f["q"].any()
    P, D, gr = oracle.gap(ref_h, (32, 32, 32), scenes.default_bins(), ref, tvl1=True)
    assert abs(stats["primal"] - P) <= 1e-4 * P
    assert abs(stats["dual"] - D) <= 1e-4 * abs(D) + 1e-3


def test_histogram_count_limit_exactly_65535(ctx):
    import paper_2107_14790_amd as tgv
    say("count limit 65535")
    sc = scenes.plane_scene(n=(3, 3, 7), z_plane_index=3, n_cams=1)
    sc.cams.vote[:] = [65535]
    _, hist = gpu_hist(ctx, sc)
    ref, mx = oracle.histograms(sc)
    assert np.array_equal(hist, ref) and mx == 65535 and hist.max() == 65535
    sc2 = scenes.plane_scene(n=(3, 3, 7), z_plane_index=3, n_cams=2)
    sc2.cams.vote[:] = [65535, 1]
    with pytest.raises(tgv.TgvError) as e:
        gpu_hist(ctx, sc2)
    assert e.value.status == tgv.TGV_E_OVERFLOW
