"""The allocation-free solve (tgv_solve_noalloc, state in the library's fixed
device workspace) against tgv_solve on the same inputs, through the C ABI:
two calls in a row, the second on a smaller block, each bit for bit equal to
the allocating entry point's fresh solve."""
import sys

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[noalloc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_14790_amd as tgv
    return tgv.Context(0)


def block(ctx, n, halo, seed):
    """Histograms of the sphere scene on an n^3 block, and a start field that
    is 0 inside and seeded values in [-1, 1] on the frozen border."""
    import paper_2107_14790_amd as tgv
    sc = scenes.sphere_scene(n=n)
    g = tgv.grid_from(sc.grid)
    g.halo = halo
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    hist = ctx.build_histograms(pyr, W, H, sc.cams, g)
    u0 = np.zeros((n, n, n), dtype=np.float32)
    if halo:
        rng = np.random.default_rng(seed)
        border = np.ones((n, n, n), dtype=bool)
        border[halo:n - halo, halo:n - halo, halo:n - halo] = False
        u0[border] = rng.uniform(-1.0, 1.0, size=int(border.sum())).astype(np.float32)
    return g, hist, torch.from_numpy(u0.reshape(-1)).cuda()


# (edge, halo, storage, iterations): the first block is large enough for the
# two-iterations-per-pass schedule, the second is smaller (one iteration per
# pass) and starts on what the first left in the workspace
CASES = [
    [(80, 0, 0, 41), (32, 2, 0, 30)],
    [(100, 0, 1, 20), (48, 1, 2, 17)],
]


@pytest.mark.parametrize("seq", CASES, ids=["f32", "f16-then-bf16"])
def test_noalloc_equals_solve_two_calls(ctx, seq):
    import paper_2107_14790_amd as tgv
    for n, halo, storage, iters in seq:
        say(f"block {n}^3 halo {halo} storage {storage} iters {iters}")
        g, hist, u0 = block(ctx, n, halo, seed=n)
        assert tgv.state_bytes(g, storage) <= tgv.NOALLOC_MAX_BYTES
        p = tgv.Params(iters=iters, storage=storage)
        u_ref = u0.clone()
        ctx.solve(g, hist, u_ref, p)
        u_na = u0.clone()
        ctx.solve_noalloc(g, hist, u_na, p)
        torch.cuda.synchronize()
        assert torch.isfinite(u_na).all()
        assert torch.equal(u_na, u_ref), float((u_na - u_ref).abs().max())
        if halo:
            # the frozen border is unchanged
            m = torch.from_numpy(np.pad(np.zeros((n - 2 * halo,) * 3, dtype=bool), halo, constant_values=True)
                                 .reshape(-1)).cuda()
            assert torch.equal(u_na[m], u0[m])


def test_noalloc_rejects_blocks_beyond_the_workspace(ctx):
    import paper_2107_14790_amd as tgv
    g = tgv.grid_c([0.0, 0.0, 0.0], 0.01, (90, 90, 90))
    assert tgv.state_bytes(g, tgv.STORE_F32) > tgv.NOALLOC_MAX_BYTES
    hist = torch.zeros((90 ** 3, 8), dtype=torch.int16, device="cuda")
    u = torch.zeros(90 ** 3, device="cuda")
    with pytest.raises(tgv.TgvError, match="fixed workspace"):
        ctx.solve_noalloc(g, hist, u, tgv.Params(iters=4))
    # nothing ran: u is untouched
    assert torch.count_nonzero(u) == 0
