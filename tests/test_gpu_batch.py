"""Batched solves of uneven blocks: each block's result is the same alone and
in the mix (bitwise), with and without the captured graph, and across
repeated graph replays with other work between them."""
import sys

import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    return tgv.Context(0)


SHAPES = [((36, 36, 36), 2), ((50, 41, 38), 2), ((70, 20, 9), 0), ((68, 68, 68), 2), ((40, 40, 72), 1),
          ((5, 6, 7), 0), ((130, 33, 34), 2)]


def make_blocks(seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for shape, halo in SHAPES:
        n = int(np.prod(shape))
        hist = np.zeros((n, 8), dtype=np.uint16)
        tot = rng.integers(0, 9, size=n)
        np.add.at(hist, (np.repeat(np.arange(n), tot), rng.integers(0, 7, size=int(tot.sum()))), 1)
        u0 = np.where(rng.random(n) < 0.5, rng.uniform(-1, 1, n), 0.0).astype(np.float32)
        out.append((shape, halo, hist, u0))
    return out


def fields(st):
    return {k: v.cpu().numpy().view(np.uint32) for k, v in st.export().items()}


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("ty", [4, 8])
def test_batch_equals_solo(ctx, storage, ty):
    import paper_2107_14790_amd as tgv
    say("batch vs solo", storage, ty)
    blocks = make_blocks(storage * 10 + ty)
    iters = 17
    solo, batch, states, hists = [], [], [], []
    for shape, halo, hist, u0 in blocks:
        g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
        h = torch.from_numpy(hist.view(np.int16)).cuda()
        u = torch.from_numpy(u0).cuda()
        a = tgv.State(ctx, g, storage)
        a.reset(u)
        ctx.solve(g, h, None, tgv.Params(iters=iters, storage=storage, tile_y=ty), state=a)
        solo.append(fields(a))
        b = tgv.State(ctx, g, storage)
        b.reset(u)
        states.append(b)
        hists.append(h)
    tz = [5, 32, 7, 16, 9, 1, 64]
    ctx.solve_batch(states, hists, tgv.Params(iters=iters, storage=storage, tile_y=ty), tile_z=tz)
    for i, st in enumerate(states):
        f = fields(st)
        for k in f:
            assert np.array_equal(f[k], solo[i][k]), (i, k)


def test_graph_replays_match_eager(ctx):
    import paper_2107_14790_amd as tgv
    say("graph replays")
    blocks = make_blocks(3)

    def run(flags, chunks):
        states, hists = [], []
        for shape, halo, hist, u0 in blocks:
            g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
            s = tgv.State(ctx, g, 0)
            s.reset(torch.from_numpy(u0).cuda())
            states.append(s)
            hists.append(torch.from_numpy(hist.view(np.int16)).cuda())
        outs = []
        for c in chunks:
            ctx.solve_batch(states, hists, tgv.Params(iters=c, flags=flags))
            torch.cuda.synchronize()
            # unrelated eager work between replays
            junk = torch.randn(1 << 20, device="cuda")
            junk.mul_(2).sum().item()
            outs.append([fields(s)["u"] for s in states])
        return outs

    eager = run(0, [9, 12, 7, 12])
    graph = run(tgv.FLAG_GRAPH, [9, 12, 7, 12])
    for a, b in zip(eager, graph):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_batch_matches_oracle_on_small_block(ctx):
    import paper_2107_14790_amd as tgv
    say("batch vs oracle")
    shape, halo, hist, u0 = make_blocks(5)[0]
    g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
    s = tgv.State(ctx, g, 0)
    s.reset(torch.from_numpy(u0).cuda())
    h = torch.from_numpy(hist.view(np.int16)).cuda()
    other = tgv.State(ctx, tgv.grid_c((0, 0, 0), 1.0, (40, 40, 40), 2), 0)
    other.reset(torch.zeros(40 ** 3, device="cuda"))
    ho = torch.zeros((40 ** 3, 8), dtype=torch.int16, device="cuda")
    ctx.solve_batch([other, s], [ho, h], tgv.Params(iters=80, flags=tgv.FLAG_GRAPH))
    u = s.export()["u"].cpu().numpy().astype(np.float64)
    ref = oracle.solve(hist, shape, scenes.default_bins(), 80, halo=halo, u0=u0.astype(np.float64))
    assert np.abs(u - ref.u).max() <= 1e-4
