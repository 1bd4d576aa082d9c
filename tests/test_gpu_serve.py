"""Served blocks on the GPU: each result is bit-identical to the same block
solved alone, while many blocks of different sizes overlap on the device."""
import sys

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_served_results_equal_solo_solves():
    import paper_2107_14790_amd as tgv
    from paper_2107_14790_amd.serve import GpuBackend, Request, Server, latency_stats, poisson_arrivals
    say("serve vs solo")
    ctx = tgv.Context(0)
    sc = scenes.sphere_scene(n=64)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    rng = np.random.default_rng(1)
    h = sc.grid.h
    t = poisson_arrivals(2000.0, 24, seed=2)
    reqs = []
    for i in range(24):
        e = int(rng.integers(12, 25)) + 4
        c = rng.uniform(-0.9, 0.9, size=3)
        g = scenes.Grid((c - 0.5 * e * h).astype(np.float32), h, (e, e + 1, e + 2), 2)
        reqs.append(Request(i, g, float(t[i]), 40))
    params = tgv.Params(iters=40)
    be = GpuBackend(ctx, pyr, W, H, sc.cams, params=params)
    srv = Server(be, budget_bytes=8 << 30, tick_iters=10)
    res = srv.run(reqs)
    assert all(r.ok for r in res), [r.error for r in res if not r.ok]
    assert srv.max_active_seen >= 2
    st = latency_stats(res)
    assert st["n_ok"] == 24
    for r in res:
        g = tgv.grid_from(reqs[r.rid].grid)
        hist = ctx.build_histograms(pyr, W, H, sc.cams, g)
        u = torch.zeros(g.nx * g.ny * g.nz, device="cuda")
        ctx.solve(g, hist, u, tgv.Params(iters=40))
        torch.cuda.synchronize()
        assert torch.equal(u, r.output), r.rid


@pytest.mark.parametrize("two", [True, False], ids=["two-per-launch", "one-per-launch"])
def test_served_city_blocks_equal_solo_solves(two):
    """The serving workload's own blocks (city scene, edges 32..192 plus a
    2-voxel halo, 500 iterations in ticks of 50, graph replay), arriving as a
    Poisson stream: each served result equals the block's solo solve bit for
    bit, whatever else was in flight."""
    import paper_2107_14790_amd as tgv
    from paper_2107_14790_amd.serve import GpuBackend, Request, Server, poisson_arrivals
    say("serve city blocks, two iterations per launch:", two)
    sc, _ = scenes.city_scene(device="cuda")
    ctx = tgv.Context(0)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    pool = scenes.city_blocks(sc, n_blocks=10, e_min=32, e_max=192, seed=5)
    if two:
        params = tgv.Params(iters=500, schedule=tgv.SCHED_FUSED2, flags=tgv.FLAG_GRAPH)
    else:
        params = tgv.Params(iters=500, schedule=tgv.SCHED_FUSED, tile_y=4, flags=tgv.FLAG_GRAPH)
    t = poisson_arrivals(40.0, len(pool), seed=7)
    reqs = [Request(i, pool[i], float(t[i]), 500) for i in range(len(pool))]
    be = GpuBackend(ctx, pyr, W, H, sc.cams, params=params)
    srv = Server(be, budget_bytes=200 << 30, tick_iters=50)
    res = srv.run(reqs)
    assert all(r.ok for r in res), [r.error for r in res if not r.ok]
    assert srv.max_active_seen >= 2
    say("served", len(res), "blocks in", srv.ticks, "ticks, at most", srv.max_active_seen, "at once")
    for r in res:
        g = tgv.grid_from(reqs[r.rid].grid)
        hist = ctx.build_histograms(pyr, W, H, sc.cams, g)
        u = torch.zeros(g.nx * g.ny * g.nz, device="cuda")
        ctx.solve(g, hist, u, tgv.Params(iters=500, schedule=params.schedule, tile_y=params.tile_y))
        torch.cuda.synchronize()
        assert torch.equal(u, r.output), r.rid
