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


def test_batch_with_block_beyond_tiled_offsets_and_table_growth(ctx):
    """A graph-replayed batch of one block, then a batch that adds a 448^3
    block (too large for the tiled kernels' 32-bit offsets: it runs its own
    per-voxel fused launches) with the same tiled work, which grows the
    block table under an otherwise identical graph.  Every block's state
    equals its solo solve bit for bit."""
    import paper_2107_14790_amd as tgv
    say("batch with a 448^3 block")
    shape_s, halo_s, hist_s, u0_s = make_blocks(3)[0]
    big = (448, 448, 448)
    nb = int(np.prod(big))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(449)
    hist_b = torch.zeros((nb, 8), dtype=torch.int16, device="cuda")
    hist_b[:, :7] = torch.randint(0, 3, (nb, 7), device="cuda", dtype=torch.int16, generator=gen)
    hist_b[torch.rand(nb, device="cuda", generator=gen) < 0.6] = 0
    u0_b = torch.zeros(nb, device="cuda")
    g_s = tgv.grid_c((0, 0, 0), 1.0, shape_s, halo_s)
    g_b = tgv.grid_c((0, 0, 0), 1.0, big, 0)
    h_s = torch.from_numpy(hist_s.view(np.int16)).cuda()
    p = tgv.Params(iters=6, flags=tgv.FLAG_GRAPH)

    def new_state(g, u0):
        st = tgv.State(ctx, g, 0)
        st.reset(u0)
        return st

    a = new_state(g_s, torch.from_numpy(u0_s).cuda())
    ctx.solve_batch([a], [h_s], p)  # captures the graph with a one-block table
    b_small = new_state(g_s, torch.from_numpy(u0_s).cuda())
    b_big = new_state(g_b, u0_b)
    ctx.solve_batch([b_small, b_big], [h_s, hist_b], p)  # same tiled work, larger table
    torch.cuda.synchronize()
    solo_s = new_state(g_s, torch.from_numpy(u0_s).cuda())
    ctx.solve(g_s, h_s, None, tgv.Params(iters=6), state=solo_s)
    solo_b = new_state(g_b, u0_b)
    ctx.solve(g_b, hist_b, None, tgv.Params(iters=6), state=solo_b)
    torch.cuda.synchronize()
    fa, fs = fields(a), fields(solo_s)
    for k in fa:
        assert np.array_equal(fa[k], fs[k]), ("first batch", k)
    fb = fields(b_small)
    for k in fb:
        assert np.array_equal(fb[k], fs[k]), ("second batch, small block", k)
    xb, yb = b_big.export(), solo_b.export()
    for k in xb:
        assert torch.equal(xb[k], yb[k]), ("second batch, 448^3 block", k)
    del xb, yb
    for st in (a, b_small, b_big, solo_s, solo_b):
        st.close()


@pytest.mark.parametrize("storage", [0, 1, 2])
@pytest.mark.parametrize("iters", [2, 9, 16])
def test_two_iteration_batch_equals_solo(ctx, storage, iters):
    """The default batched solve (two iterations per persistent launch, an
    odd leftover pass as one batched one-iteration launch) against each block
    solved alone with the one-iteration kernel, in every storage precision."""
    import paper_2107_14790_amd as tgv
    say("two-iteration batch vs solo", storage, iters)
    blocks = make_blocks(100 + storage)
    solo, states, hists = [], [], []
    for shape, halo, hist, u0 in blocks:
        g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
        h = torch.from_numpy(hist.view(np.int16)).cuda()
        u = torch.from_numpy(u0).cuda()
        a = tgv.State(ctx, g, storage)
        a.reset(u)
        ctx.solve(g, h, None, tgv.Params(iters=iters, storage=storage, schedule=tgv.SCHED_FUSED), state=a)
        solo.append(fields(a))
        b = tgv.State(ctx, g, storage)
        b.reset(u)
        states.append(b)
        hists.append(h)
    ctx.solve_batch(states, hists, tgv.Params(iters=iters, storage=storage))
    for i, st in enumerate(states):
        f = fields(st)
        for k in f:
            assert np.array_equal(f[k], solo[i][k]), (i, k)


def test_autotuned_batch_equals_solo(ctx):
    """The autotuner's pick (schedule, tile_y, per-block tile_z, timed on this
    GPU) runs the batch; every block's state equals its solo solve with the
    library's defaults, bit for bit."""
    import paper_2107_14790_amd as tgv
    from paper_2107_14790_amd.autotune import Autotuner
    say("autotuned batch")
    blocks = make_blocks(7)
    grids = [tgv.grid_c((0, 0, 0), 1.0, shape, halo) for shape, halo, _, _ in blocks]

    class Gn:
        def __init__(self, n):
            self.n = n

    tuned = Autotuner(ctx, iters=5, reps=1).tune([Gn(shape) for shape, _, _, _ in blocks])
    say("tuned", tuned["schedule"], tuned["tile_y"], tuned["tile_z"], tuned["checked_on_batch"])
    assert tuned["tile_z"] is None or len(tuned["tile_z"]) == len(blocks)
    assert tuned["checked_on_batch"]["chosen"] in tuned["checked_on_batch"]["ms"]
    iters = 12
    solo, states, hists = [], [], []
    for (shape, halo, hist, u0), g in zip(blocks, grids):
        h = torch.from_numpy(hist.view(np.int16)).cuda()
        u = torch.from_numpy(u0).cuda()
        a = tgv.State(ctx, g)
        a.reset(u)
        ctx.solve(g, h, None, tgv.Params(iters=iters), state=a)
        solo.append(fields(a))
        b = tgv.State(ctx, g)
        b.reset(u)
        states.append(b)
        hists.append(h)
    p = Autotuner.params(tuned, iters, flags=tgv.FLAG_GRAPH)
    ctx.solve_batch(states, hists, p, tile_z=tuned["tile_z"])
    for i, st in enumerate(states):
        f = fields(st)
        for k in f:
            assert np.array_equal(f[k], solo[i][k]), (i, k)


def test_two_iteration_batch_with_a_state_beyond_one_descriptor(ctx):
    """A float32 batch whose 280^3 block has a state of more than 2 GiB (no
    single buffer descriptor reaches all its fields), with two small blocks:
    the whole batch then runs the batched kernel with one descriptor per
    field; every block equals its solo solve bit for bit."""
    import paper_2107_14790_amd as tgv
    say("two-iteration batch with a state beyond 2 GiB")
    big = (280, 280, 280)
    assert tgv.state_bytes(tgv.grid_c((0, 0, 0), 1.0, big, 0), 0) > (1 << 31)
    nb = int(np.prod(big))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(281)
    hist_b = torch.zeros((nb, 8), dtype=torch.int16, device="cuda")
    hist_b[:, :7] = torch.randint(0, 3, (nb, 7), device="cuda", dtype=torch.int16, generator=gen)
    u0_b = torch.where(torch.rand(nb, device="cuda", generator=gen) < 0.5,
                       torch.rand(nb, device="cuda", generator=gen) * 2 - 1, torch.zeros(nb, device="cuda"))
    small = make_blocks(11)[:2]
    grids = [tgv.grid_c((0, 0, 0), 1.0, shape, halo) for shape, halo, _, _ in small]
    grids.append(tgv.grid_c((0, 0, 0), 1.0, big, 0))
    hists = [torch.from_numpy(h.view(np.int16)).cuda() for _, _, h, _ in small] + [hist_b]
    u0s = [torch.from_numpy(u0).cuda() for _, _, _, u0 in small] + [u0_b]
    iters = 5
    states = []
    for g, u0 in zip(grids, u0s):
        st = tgv.State(ctx, g, 0)
        st.reset(u0)
        states.append(st)
    ctx.solve_batch(states, hists, tgv.Params(iters=iters))
    for i, (g, h, u0) in enumerate(zip(grids, hists, u0s)):
        solo = tgv.State(ctx, g, 0)
        solo.reset(u0)
        ctx.solve(g, h, None, tgv.Params(iters=iters, schedule=tgv.SCHED_FUSED), state=solo)
        xb, ys = states[i].export(), solo.export()
        for k in xb:
            assert torch.equal(xb[k], ys[k]), (i, k)
        del xb, ys
        solo.close()
    for st in states:
        st.close()
