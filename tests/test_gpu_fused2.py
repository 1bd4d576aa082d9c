"""Two fused iterations per pass (schedule FUSED2) against one per pass.

The temporal-blocked kernel evaluates the same per-voxel arithmetic as the
one-iteration kernel, only in a different order over the grid, so the whole
solver state after a solve (u, v, the previous primal iterate, p, q) must be
bit-identical for every shape, tile, storage precision, model and iteration
count, including odd counts (one single pass left over) and the ragged
edges of tiles in x, y and z."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print("[fused2]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    c = tgv.Context(0)
    yield c
    c.close()


def random_problem(shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    hist = np.zeros((n, 8), dtype=np.uint16)
    tot = rng.integers(0, 12, size=n)
    for x in np.nonzero(tot)[0]:
        hist[x, :7] = np.bincount(rng.integers(0, 7, size=tot[x]), minlength=7)
    u0 = np.where(rng.random(n) < 0.5, rng.uniform(-1, 1, n), 0.0).astype(np.float32)
    return hist, u0


def run(ctx, shape, hist_np, u0_np, halo, params):
    import paper_2107_14790_amd as tgv
    g = tgv.grid_c((0, 0, 0), 1.0, shape, halo)
    n = int(np.prod(shape))
    hist = torch.from_numpy(hist_np.view(np.int16).reshape(n, 8)).cuda()
    st = tgv.State(ctx, g, storage=params.storage)
    st.reset(torch.from_numpy(u0_np).cuda())
    ctx.solve(g, hist, None, params, state=st)
    f = st.export()
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in f.items()}
    st.close()
    return out


def assert_same_state(a, b):
    for k in ("u", "v", "u_prev", "v_prev", "p", "q"):
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k


CASES = [
    # shape, halo, iters, tile_y, tile_z
    ((70, 9, 5), 0, 9, 4, 2),
    ((37, 29, 23), 2, 20, 4, 5),
    ((37, 29, 23), 2, 21, 6, 64),
    ((130, 21, 40), 0, 12, 4, 7),
    ((130, 21, 40), 0, 13, 6, 1),
    ((64, 8, 8), 3, 6, 4, 3),
    ((65, 7, 67), 1, 4, 6, 16),
    ((1, 1, 1), 0, 5, 4, 1),
    ((17, 1, 1), 0, 8, 4, 2),
    ((1, 13, 6), 0, 7, 6, 3),
    ((3, 2, 2), 0, 3, 4, 1),
    ((100, 45, 33), 1, 9, 7, 13),
    ((64, 7, 20), 0, 6, 7, 64),
    ((130, 50, 41), 2, 10, 7, 9),
]


@pytest.mark.parametrize("shape,halo,iters,ty,cz", CASES)
def test_fused2_state_bit_identical(ctx, shape, halo, iters, ty, cz):
    import paper_2107_14790_amd as tgv
    say("shape", shape, "halo", halo, "iters", iters, "tile", ty, cz)
    hist, u0 = random_problem(shape, sum(shape) * 7 + iters)
    ref = run(ctx, shape, hist, u0, halo, tgv.Params(iters=iters, schedule=tgv.SCHED_FUSED))
    got = run(ctx, shape, hist, u0, halo, tgv.Params(iters=iters, schedule=tgv.SCHED_FUSED2, tile_y=ty, tile_z=cz))
    assert_same_state(ref, got)


@pytest.mark.parametrize("storage", [1, 2])
def test_fused2_low_precision_storage_bit_identical(ctx, storage):
    import paper_2107_14790_amd as tgv
    shape = (100, 19, 33)
    say("storage", storage, shape)
    hist, u0 = random_problem(shape, 11 + storage)
    ref = run(ctx, shape, hist, u0, 1, tgv.Params(iters=11, storage=storage, schedule=tgv.SCHED_FUSED))
    got = run(ctx, shape, hist, u0, 1, tgv.Params(iters=11, storage=storage, schedule=tgv.SCHED_FUSED2, tile_z=6))
    assert_same_state(ref, got)


def test_fused2_tvl1_bit_identical(ctx):
    import paper_2107_14790_amd as tgv
    shape = (70, 30, 18)
    say("tvl1", shape)
    hist, u0 = random_problem(shape, 5)
    ref = run(ctx, shape, hist, u0, 0, tgv.Params(iters=10, flags=tgv.FLAG_TVL1, schedule=tgv.SCHED_FUSED))
    got = run(ctx, shape, hist, u0, 0, tgv.Params(iters=10, flags=tgv.FLAG_TVL1, schedule=tgv.SCHED_FUSED2,
                                                   tile_y=6, tile_z=4))
    assert_same_state(ref, got)


def test_fused2_rejects_unsupported_tile(ctx):
    import paper_2107_14790_amd as tgv
    shape = (8, 8, 8)
    hist, u0 = random_problem(shape, 1)
    with pytest.raises(tgv.TgvError) as e:
        run(ctx, shape, hist, u0, 0, tgv.Params(iters=4, schedule=tgv.SCHED_FUSED2, tile_y=8))
    assert e.value.status == tgv.TGV_E_INVAL


def test_fused2_terrain256_sampled_state(ctx):
    """The bench's block (256^3) in the bench's launch shape: one and two
    iterations per pass (and the default schedule, which picks the latter
    at this size) agree bit for bit on the whole state."""
    import paper_2107_14790_amd as tgv
    shape = (256, 256, 256)
    say("256^3 default tiles")
    rng = np.random.default_rng(256)
    n = int(np.prod(shape))
    hist = np.zeros((n, 8), dtype=np.uint16)
    hist[:, :7] = rng.integers(0, 3, size=(n, 7), dtype=np.uint16) * (rng.random((n, 1)) < 0.3)
    u0 = np.zeros(n, np.float32)
    ref = run(ctx, shape, hist, u0, 0, tgv.Params(iters=7, schedule=tgv.SCHED_FUSED))
    got = run(ctx, shape, hist, u0, 0, tgv.Params(iters=7, schedule=tgv.SCHED_FUSED2))
    auto = run(ctx, shape, hist, u0, 0, tgv.Params(iters=7))  # the default picks FUSED2 here
    assert_same_state(ref, auto)
    assert_same_state(ref, got)


@pytest.mark.parametrize("storage", [0, 1])
def test_fused2_tvl1_default_tile_bit_identical(ctx, storage):
    """TV-L1 with the default 64 x 7 tile (in float32 its own kernel, which
    moves no v or q) against one iteration per pass."""
    import paper_2107_14790_amd as tgv
    shape = (130, 21, 40)
    say("tvl1 default tile", shape, "storage", storage)
    hist, u0 = random_problem(shape, 77 + storage)
    ref = run(ctx, shape, hist, u0, 1, tgv.Params(iters=13, storage=storage, flags=tgv.FLAG_TVL1,
                                                   schedule=tgv.SCHED_FUSED))
    got = run(ctx, shape, hist, u0, 1, tgv.Params(iters=13, storage=storage, flags=tgv.FLAG_TVL1,
                                                   schedule=tgv.SCHED_FUSED2))
    assert_same_state(ref, got)
    assert not got["v"].any() and not got["q"].any()


def test_tvl1_after_tgv_sets_v_and_q_to_zero(ctx):
    """A TV-L1 solve of a state that holds a TGV iterate starts by setting v
    and q to 0 (Eq. 1 has neither), on every schedule alike."""
    import paper_2107_14790_amd as tgv
    shape = (70, 30, 18)
    hist_np, u0_np = random_problem(shape, 91)
    n = int(np.prod(shape))
    g = tgv.grid_c((0, 0, 0), 1.0, shape, 0)
    hist = torch.from_numpy(hist_np.view(np.int16).reshape(n, 8)).cuda()
    out = []
    for sched in (tgv.SCHED_FUSED, tgv.SCHED_FUSED2, tgv.SCHED_SPLIT):
        st = tgv.State(ctx, g)
        st.reset(torch.from_numpy(u0_np).cuda())
        ctx.solve(g, hist, None, tgv.Params(iters=10, schedule=sched), state=st)
        mid = st.export()
        ctx.solve(g, hist, None, tgv.Params(iters=9, schedule=sched, flags=tgv.FLAG_TVL1), state=st)
        f = {k: v.cpu().numpy() for k, v in st.export().items()}
        st.close()
        assert mid["v"].abs().max().item() > 0 and mid["q"].abs().max().item() > 0
        assert not f["v"].any() and not f["v_prev"].any() and not f["q"].any()
        out.append(f)
    assert_same_state(out[0], out[1])
    assert_same_state(out[0], out[2])


def test_fused2_on_caller_memory_and_a_large_state(ctx):
    """The two-iteration kernel on a state in caller memory (a torch tensor,
    as the server uses) and on a 2.2 GiB float32 state (beyond the one-
    descriptor form) equals one iteration per pass."""
    import paper_2107_14790_amd as tgv
    for shape, wrapped in (((130, 50, 41), True), ((272, 272, 288), False)):
        say("caller memory" if wrapped else "state above 2 GiB", shape)
        n = int(np.prod(shape))
        g = tgv.grid_c((0, 0, 0), 1.0, shape, 0)
        rng = np.random.default_rng(n % 1000)
        hist = torch.zeros((n, 8), dtype=torch.int16, device="cuda")
        hist[:, :7] = torch.from_numpy(rng.integers(0, 3, size=(n, 7)).astype(np.int16)).cuda()
        outs = []
        for sched in (tgv.SCHED_FUSED, tgv.SCHED_FUSED2):
            mem = torch.empty(tgv.state_bytes(g) // 4 + 64, dtype=torch.float32, device="cuda") if wrapped else None
            st = tgv.State(ctx, g, memory=mem)
            assert (st.bytes() > (1 << 31)) == (not wrapped)
            st.reset(torch.zeros(n, device="cuda"))
            ctx.solve(g, hist, None, tgv.Params(iters=4, schedule=sched), state=st)
            outs.append(st.export()["u"].cpu())
            st.close()
            del mem
        assert torch.equal(outs[0].view(torch.int32), outs[1].view(torch.int32))
