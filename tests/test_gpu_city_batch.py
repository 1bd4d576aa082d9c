"""Parity of the batched solve at the batching workload's full size.

The city workload (512 blocks of uneven size, interior edges log-uniform in
32..128 plus a 2-voxel frozen halo, 256 oblique 1024x1024 depth maps, 500
iterations) is solved the way the benchmark times it: every block in one
batched solve, two iterations per persistent launch, replayed from a HIP
graph.  A seeded random sample of 16 blocks is then checked against the
oracle one by one: histograms bit for bit, u after 500 iterations within
1e-4 of the float64 solve.  The oracle runs its per-voxel loops on the host's
cores (bit-identical to its serial form), which keeps the sample (about
4.5e9 updates) to well under a minute."""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu

ITERS = 500
SAMPLE = 16


def say(*a):
    print("[city]", *a, flush=True)
    sys.stdout.flush()


def host_threads():
    return max(1, min(16, os.cpu_count() or 1))


def test_city_batch_sampled_blocks_match_oracle():
    import paper_2107_14790_amd as tgv
    if not os.path.exists(scenes._RAYLIB):
        scenes.build_raycaster()
    t0 = time.perf_counter()
    sc, _ = scenes.city_scene(device="cuda")
    grids = scenes.city_blocks(sc)
    say(f"scene and {len(grids)} blocks in {time.perf_counter() - t0:.1f} s")
    ctx = tgv.Context(0)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    cams = tgv.cameras_from(sc.cams)
    hists, states = [], []
    for g in grids:
        gc = tgv.grid_from(g)
        hists.append(ctx.build_histograms(pyr, W, H, cams, gc))
        st = tgv.State(ctx, gc, 0)
        st.reset(torch.zeros(gc.nx * gc.ny * gc.nz, device="cuda"))
        states.append(st)
    params = tgv.Params(iters=ITERS, schedule=tgv.SCHED_FUSED2, flags=tgv.FLAG_GRAPH)
    ctx.solve_batch(states, hists, params)
    torch.cuda.synchronize()
    say("batched solve done")

    rng = np.random.default_rng(4004)
    pick = sorted(rng.choice(len(grids), size=SAMPLE, replace=False).tolist())
    edges = sorted({grids[i].n[0] for i in pick})
    assert min(edges) <= 64 < max(edges)  # one and two tiles across
    with oracle.threads(host_threads()):
        opyr = oracle.pyramids(sc.depth)
        for i in pick:
            g = grids[i]
            shape = tuple(int(v) for v in g.n)
            t = time.perf_counter()
            ref_h, _ = oracle.histograms(scenes.Scene(sc.depth, sc.cams, g), opyr)
            got_h = hists[i].cpu().numpy().view(np.uint16).reshape(-1, 8)
            assert np.array_equal(got_h, ref_h), f"block {i} histograms"
            assert ref_h[:, :7].sum() > 0
            st = oracle.solve(ref_h, shape, scenes.default_bins(), ITERS, halo=g.halo)
            u = states[i].export()["u"].cpu().numpy().astype(np.float64)
            err = np.abs(u - st.u).max()
            say(f"block {i} {shape} h={g.h:.5f}: max|u - u_oracle| = {err:.2e} "
                f"({time.perf_counter() - t:.1f} s)")
            assert err <= 1e-4, i
    for st in states:
        st.close()
    ctx.close()
