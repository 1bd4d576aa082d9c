"""Calls of one context on two streams.

The context owns a few buffers that consecutive calls reuse: the culled
camera table of the histogram build, the block and tile tables (and queue
counters) of a batched solve, and the state of a solve given none.  Calls
issued back to back on two streams must still give the results of the same
calls made one after another on one stream, bit for bit."""
import sys

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[streams]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    c = tgv.Context(0)
    yield c
    c.close()


def random_hist(shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    h = np.zeros((n, 8), dtype=np.uint16)
    h[:, :7] = rng.integers(0, 3, size=(n, 7), dtype=np.uint16) * (rng.random((n, 1)) < 0.4)
    return torch.from_numpy(h.view(np.int16)).cuda()


def test_histograms_on_two_streams(ctx):
    import paper_2107_14790_amd as tgv
    scs = [scenes.sphere_scene(n=48), scenes.sphere_scene(seed=2, n_cams=5, n=40, ring_radius=2.5)]
    ins = []
    for sc in scs:
        H, W = sc.depth.shape[1:]
        ins.append((ctx.build_pyramids(torch.from_numpy(sc.depth).cuda()), W, H))
    refs = [ctx.build_histograms(p, W, H, sc.cams, tgv.grid_from(sc.grid)) for sc, (p, W, H) in zip(scs, ins)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(4):
        say("histograms, round", rep)
        outs = []
        for sc, (p, W, H), s in zip(scs, ins, streams):
            with torch.cuda.stream(s):
                outs.append(ctx.build_histograms(p, W, H, sc.cams, tgv.grid_from(sc.grid)))
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)


@pytest.mark.parametrize("graph", [False, True])
def test_batched_solves_on_two_streams(ctx, graph):
    import paper_2107_14790_amd as tgv
    shapes = [(96, 80, 72), (50, 37, 41), (70, 66, 33)]
    grids = [tgv.grid_c((0, 0, 0), 1.0, s, 1) for s in shapes]
    hists = [random_hist(s, 31 + i) for i, s in enumerate(shapes)]
    flags = tgv.FLAG_GRAPH if graph else 0
    params = tgv.Params(iters=9, schedule=tgv.SCHED_FUSED2, flags=flags)
    groups = [[0, 1], [2]]

    def fresh():
        sts = [tgv.State(ctx, g) for g in grids]
        for st, g in zip(sts, grids):
            st.reset(torch.zeros(g.nx * g.ny * g.nz, device="cuda"))
        return sts

    sts = fresh()
    for grp in groups:
        ctx.solve_batch([sts[i] for i in grp], [hists[i] for i in grp], params)
    ref = [st.export()["u"] for st in sts]
    torch.cuda.synchronize()
    for st in sts:
        st.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        say("batched, graph", graph, "round", rep)
        sts = fresh()
        torch.cuda.synchronize()
        for grp, s in zip(groups, streams):
            with torch.cuda.stream(s):
                ctx.solve_batch([sts[i] for i in grp], [hists[i] for i in grp], params)
        torch.cuda.synchronize()
        for st, r in zip(sts, ref):
            assert torch.equal(st.export()["u"], r)
        torch.cuda.synchronize()
        for st in sts:
            st.close()


def test_stateless_solves_on_two_streams(ctx):
    """Two solves without a state on the same grid share the context's
    state: the second, on another stream, waits for the first."""
    import paper_2107_14790_amd as tgv
    shape = (120, 64, 48)
    g = tgv.grid_c((0, 0, 0), 1.0, shape, 0)
    ha, hb = random_hist(shape, 7), random_hist(shape, 8)
    n = int(np.prod(shape))
    params = tgv.Params(iters=12)
    refs = []
    for h in (ha, hb):
        u = torch.zeros(n, device="cuda")
        ctx.solve(g, h, u, params)
        refs.append(u)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        say("stateless, round", rep)
        us = [torch.zeros(n, device="cuda") for _ in range(2)]
        torch.cuda.synchronize()
        for h, u, s in zip((ha, hb), us, streams):
            with torch.cuda.stream(s):
                ctx.solve(g, h, u, params)
        torch.cuda.synchronize()
        for u, r in zip(us, refs):
            assert torch.equal(u, r)
