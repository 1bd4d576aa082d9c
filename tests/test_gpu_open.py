"""Open states (TGV_FLAG_LEAVE_OPEN): a solve cut into calls that leave the
state open between them, then closed, equals one uninterrupted solve bit for
bit, for single states on every schedule and for batches that mix open and
closed states (two iterations per launch with odd pass counts, 64 x 6 and
64 x 7 tables, one iteration per launch, graph replay); an open state
cannot be exported, evaluated or continued with another model."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print("[open]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    return tgv.Context(0)


SHAPES = [((36, 36, 36), 2), ((70, 20, 9), 0), ((68, 68, 68), 2), ((40, 40, 72), 1), ((5, 6, 7), 0)]


def make_blocks(seed):
    rng = np.random.default_rng(seed)
    out = []
    for shape, halo in SHAPES:
        n = int(np.prod(shape))
        hist = np.zeros((n, 8), dtype=np.uint16)
        tot = rng.integers(0, 9, size=n)
        np.add.at(hist, (np.repeat(np.arange(n), tot), rng.integers(0, 7, size=int(tot.sum()))), 1)
        u0 = np.where(rng.random(n) < 0.5, rng.uniform(-1, 1, n), 0.0).astype(np.float32)
        out.append((shape, halo, torch.from_numpy(hist.view(np.int16)).cuda(), torch.from_numpy(u0).cuda()))
    return out


def fields(st):
    return {k: v.cpu().numpy().view(np.uint32) for k, v in st.export().items()}


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


@pytest.mark.parametrize("sched", [0, 1, 2, 3])
def test_single_state_cut_into_open_calls(ctx, sched):
    import paper_2107_14790_amd as tgv
    say("single state, schedule", sched)
    shape, halo, h, u0 = make_blocks(sched)[2]
    g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
    ref = tgv.State(ctx, g)
    ref.reset(u0)
    ctx.solve(g, h, None, tgv.Params(iters=23, schedule=sched), state=ref)
    st = tgv.State(ctx, g)
    st.reset(u0)
    for k in (1, 6, 0, 9, 7):  # 23 iterations over calls that leave the state open
        ctx.solve(g, h, None, tgv.Params(iters=k, schedule=sched, flags=tgv.FLAG_LEAVE_OPEN), state=st)
    ctx.solve(g, h, None, tgv.Params(iters=0, schedule=sched), state=st)  # close
    assert same(fields(st), fields(ref))
    # a closing call that also advances: 23 = 20 open + 3 closing
    st.reset(u0)
    ctx.solve(g, h, None, tgv.Params(iters=20, schedule=sched, flags=tgv.FLAG_LEAVE_OPEN), state=st)
    ctx.solve(g, h, None, tgv.Params(iters=3, schedule=sched), state=st)
    assert same(fields(st), fields(ref))


@pytest.mark.parametrize("sched,ty,graph", [(3, 0, False), (3, 6, True), (3, 4, False), (0, 4, True), (0, 8, False)])
def test_batch_mixing_open_and_closed_states(ctx, sched, ty, graph):
    import paper_2107_14790_amd as tgv
    say("batch, schedule", sched, "tile_y", ty, "graph", graph)
    blocks = make_blocks(10 + ty)
    flags = tgv.FLAG_GRAPH if graph else 0
    # block i gets `pre[i]` iterations before the mixed batch (0: it joins closed)
    pre = [0, 4, 0, 7, 1]
    k = [5, 6]  # two mixed ticks: odd and even pass counts
    solo, states, hists, grids = [], [], [], []
    for (shape, halo, h, u0), p0 in zip(blocks, pre):
        g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
        a = tgv.State(ctx, g)
        a.reset(u0)
        ctx.solve(g, h, None, tgv.Params(iters=p0 + sum(k), tile_y=ty, schedule=sched), state=a)
        solo.append(fields(a))
        b = tgv.State(ctx, g)
        b.reset(u0)
        if p0:
            ctx.solve(g, h, None, tgv.Params(iters=p0, tile_y=ty, schedule=sched, flags=tgv.FLAG_LEAVE_OPEN), state=b)
        states.append(b)
        hists.append(h)
        grids.append(g)
    for kk in k:
        ctx.solve_batch(states, hists, tgv.Params(iters=kk, tile_y=ty, schedule=sched,
                                                  flags=flags | tgv.FLAG_LEAVE_OPEN))
    # close them all in one batched call without iterations
    ctx.solve_batch(states, hists, tgv.Params(iters=0, tile_y=ty, schedule=sched))
    for i, st in enumerate(states):
        assert same(fields(st), solo[i]), i


def test_open_state_errors(ctx):
    import paper_2107_14790_amd as tgv
    shape, halo, h, u0 = make_blocks(3)[0]
    g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
    st = tgv.State(ctx, g)
    st.reset(u0)
    ctx.solve(g, h, None, tgv.Params(iters=3, flags=tgv.FLAG_LEAVE_OPEN), state=st)
    with pytest.raises(tgv.TgvError, match="open"):
        st.export()
    with pytest.raises(tgv.TgvError, match="open"):
        ctx.energy(st, h)
    with pytest.raises(tgv.TgvError, match="model"):
        ctx.solve(g, h, None, tgv.Params(iters=2, flags=tgv.FLAG_TVL1), state=st)
    u = torch.zeros_like(u0)
    with pytest.raises(tgv.TgvError):  # an output or statistics with the flag
        ctx.solve(g, h, u, tgv.Params(iters=2, flags=tgv.FLAG_LEAVE_OPEN), state=st)
    with pytest.raises(tgv.TgvError):
        ctx.solve(g, h, None, tgv.Params(iters=2, flags=tgv.FLAG_LEAVE_OPEN), state=st, stats=True)
    with pytest.raises(tgv.TgvError):  # a fresh solve must close
        ctx.solve(g, h, u, tgv.Params(iters=2, flags=tgv.FLAG_LEAVE_OPEN))
    # closing leaves it usable; the stats are those of 3 iterations
    s = ctx.solve(g, h, None, tgv.Params(iters=0), state=st, stats=True)
    assert s["iters_done"] == 3
    ref = tgv.State(ctx, g)
    ref.reset(u0)
    ctx.solve(g, h, None, tgv.Params(iters=3), state=ref)
    assert same(fields(st), fields(ref))
