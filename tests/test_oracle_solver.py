"""Pins of the oracle's TGV-L1 solver (Eq. 1-3, primal-dual method of Sec. 3.2)
against what the mathematics fixes: operator identities, closed-form
minimisers, an exact LP in 1-D, an independent smoothed solver in 3-D and
weak duality.  CPU only."""
import numpy as np
import pytest
import torch
from scipy.optimize import linprog, minimize

import oracle
import scenes

C7 = scenes.default_bins(7, 0)
C64 = C7[:7].astype(np.float64)


def rand_hist(shape, rng, odd=True, lo=1, hi=9, fully=True):
    n = int(np.prod(shape))
    h = np.zeros((n, 8), dtype=np.uint16)
    for x in range(n):
        if not fully and rng.random() < 0.3:
            continue
        tot = int(rng.integers(lo, hi + 1))
        if odd and tot % 2 == 0:
            tot += 1
        b = rng.integers(0, 7, size=tot)
        h[x, :7] = np.bincount(b, minlength=7)
    return h


# ---------------------------------------------------------------------------
# operators (Eq. 2, Eq. 3)
# ---------------------------------------------------------------------------
def test_adjointness_random():
    rng = np.random.default_rng(1)
    shape = (5, 4, 3)
    n = 60
    u, v = rng.normal(size=n), rng.normal(size=3 * n)
    p, q = rng.normal(size=3 * n), rng.normal(size=6 * n)
    kp, kq = oracle.apply_K(u, v, shape)
    gu, gv = oracle.apply_KT(p, q, shape)
    w = np.repeat([1.0, 1.0, 1.0, 2.0, 2.0, 2.0], n)  # weighted inner product on q
    lhs = kp @ p + (w * kq) @ q
    rhs = u @ gu + v @ gv
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def test_K_closed_forms():
    nx, ny, nz = 6, 5, 4
    n = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    # u = x^2, v = 0: forward difference 2x + 1 except the last x-cell (dropped)
    kp, kq = oracle.apply_K((x ** 2).astype(float), np.zeros(3 * n), (nx, ny, nz))
    np.testing.assert_array_equal(kp[:n], np.where(x < nx - 1, 2 * x + 1, 0))
    assert not kp[n:].any() and not kq.any()
    # u = 0, v_x = y: E_xy = d-_y v_x / 2 = 1/2 where y > 0
    v = np.zeros(3 * n)
    v[:n] = y
    kp, kq = oracle.apply_K(np.zeros(n), v, (nx, ny, nz))
    np.testing.assert_array_equal(kq[3 * n:4 * n], np.where(y > 0, 0.5, 0.0))
    assert not kq[:3 * n].any() and not kq[4 * n:].any()
    np.testing.assert_array_equal(kp[:n], np.where(x < nx - 1, -y, 0))
    # v_z = z^2: E_zz = z^2 - (z-1)^2 = 2z - 1 where z > 0
    v = np.zeros(3 * n)
    v[2 * n:] = z ** 2
    kp, kq = oracle.apply_K(np.zeros(n), v, (nx, ny, nz))
    np.testing.assert_array_equal(kq[2 * n:3 * n], np.where(z > 0, 2 * z - 1, 0))


def test_affine_u_with_matching_v_has_zero_K():
    nx, ny, nz = 7, 6, 5
    n = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c, d = 0.375, -0.25, 0.125, 0.5
    u = (a * x + b * y + c * z + d).ravel()
    v = np.concatenate([np.full(n, a), np.full(n, b), np.full(n, c)])
    kp, kq = oracle.apply_K(u, v, (nx, ny, nz))
    assert not kp.any() and not kq.any()


def test_operator_norm_bound():
    L2 = oracle.norm_K2((12, 12, 12), iters=400)
    assert 15.0 < L2 <= 16.0 + 1e-9


# ---------------------------------------------------------------------------
# proximal map of the histogram data term
# ---------------------------------------------------------------------------
def _prox_obj(w, ut, hk, ck, tau, lam):
    return (w - ut) ** 2 / (2 * tau) + lam * np.sum(hk[None, :] * np.abs(w[:, None] - ck[None, :]), axis=1)


def test_prox_against_dense_search():
    rng = np.random.default_rng(2)
    grid = np.linspace(-4, 4, 160001)
    for _ in range(300):
        hk = rng.integers(0, 6, size=7).astype(float)
        ut = rng.uniform(-3, 3)
        tau, lam = rng.uniform(0.05, 1.0), rng.uniform(0.0, 2.0)
        w = oracle.prox(ut, hk, C64, tau, lam)
        vals = _prox_obj(grid, ut, hk, C64, tau, lam)
        wg = grid[np.argmin(vals)]
        assert abs(w - wg) <= 6e-5
        assert _prox_obj(np.array([w]), ut, hk, C64, tau, lam)[0] <= vals.min() + 1e-12


def test_prox_limits():
    rng = np.random.default_rng(3)
    for _ in range(100):
        hk = rng.integers(0, 6, size=7).astype(float)
        if hk.sum() % 2 == 0:
            hk[3] += 1
        ut = rng.uniform(-3, 3)
        assert oracle.prox(ut, hk, C64, 0.3, 0.0) == ut          # no data weight: identity
        lo, hi = oracle.weighted_median_interval(hk.astype(int), C64)
        assert oracle.prox(ut, hk, C64, 1e6, 1.0) == lo          # huge step: the weighted median
    assert oracle.prox(0.7, np.zeros(7), C64, 0.3, 1.0) == 0.7   # empty histogram


# ---------------------------------------------------------------------------
# solver special cases
# ---------------------------------------------------------------------------
def test_alpha_zero_gives_weighted_median():
    rng = np.random.default_rng(4)
    shape = (6, 5, 4)
    hist = rand_hist(shape, rng, odd=True)
    st = oracle.solve(hist, shape, C7, 200, alpha0=0.0, alpha1=0.0)
    med = np.array([oracle.weighted_median_interval(hist[x, :7].astype(int), C64)[0] for x in range(hist.shape[0])])
    np.testing.assert_array_equal(st.u, med)
    assert not st.p.any() and not st.q.any()


def test_constant_histograms_give_constant_median():
    shape = (6, 5, 4)
    n = 120
    hist = np.zeros((n, 8), dtype=np.uint16)
    hist[:, :7] = [0, 1, 0, 2, 4, 0, 0]  # W = 7, weighted median = c_4 = 1/3
    st = oracle.solve(hist, shape, C7, 400)
    np.testing.assert_allclose(st.u, np.float32(C7[4]), atol=1e-9)


def test_affine_plane_reproduced_through_histogram_path():
    # plane at voxel index 3 along z seen head-on: the histogram of voxel k
    # concentrates at c_{6-k}, i.e. u = 1 - k/3, an affine field of zero TGV
    # energy; it is the unique minimiser, so the solver must return it
    sc = scenes.plane_scene(n=(4, 3, 7), z_plane_index=3, n_cams=5)
    hist, _ = oracle.histograms(sc)
    H = hist.reshape(7, 3, 4, 8)
    for k in range(7):
        assert H[k, :, :, 6 - k].min() == 5 and H[k].sum() == 5 * 12
    shape = (4, 3, 7)
    st = oracle.solve(hist, shape, C7, 3000)
    u = st.u.reshape(7, 3, 4)
    expect = np.array([np.float64(C7[6 - k]) for k in range(7)])
    np.testing.assert_allclose(u, np.broadcast_to(expect[:, None, None], u.shape), atol=1e-6)
    P, parts = oracle.primal_energy(hist, shape, C7, st.u, st.v)
    assert P < 1e-5


def test_frozen_halo_and_bitwise_resume():
    rng = np.random.default_rng(5)
    shape = (8, 7, 6)
    n = 336
    hist = rand_hist(shape, rng, fully=False)
    u0 = rng.uniform(-1, 1, size=n)
    a = oracle.solve(hist, shape, C7, 60, halo=2, u0=u0)
    b = oracle.solve(hist, shape, C7, 25, halo=2, u0=u0)
    b = oracle.solve(hist, shape, C7, 35, halo=2, state=b)
    for k in ("u", "v", "p", "q", "ubar", "vbar"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k))
    z, y, x = np.meshgrid(np.arange(6), np.arange(7), np.arange(8), indexing="ij")
    frozen = ((x < 2) | (x >= 6) | (y < 2) | (y >= 5) | (z < 2) | (z >= 4)).ravel()
    np.testing.assert_array_equal(a.u[frozen], u0[frozen])
    assert np.any(a.u[~frozen] != u0[~frozen])


@pytest.mark.parametrize("tvl1", [False, True])
def test_threaded_oracle_is_bitwise_the_serial_one(tvl1):
    """The per-voxel sweeps split over threads give the serial iterates bit
    for bit (each voxel's update reads only the previous sweep's arrays)."""
    rng = np.random.default_rng(17)
    shape = (23, 17, 11)
    hist = rand_hist(shape, rng, fully=False)
    u0 = np.where(rng.random(int(np.prod(shape))) < 0.5, rng.uniform(-1, 1, int(np.prod(shape))), 0.0)
    ref = oracle.solve(hist, shape, C7, 40, halo=1, u0=u0, tvl1=tvl1)
    for k in (2, 5):
        with oracle.threads(k):
            assert oracle.get_threads() == k
            got = oracle.solve(hist, shape, C7, 40, halo=1, u0=u0, tvl1=tvl1)
        assert oracle.get_threads() == 1
        for f in ("u", "v", "p", "q", "ubar", "vbar"):
            assert np.array_equal(getattr(ref, f).view(np.uint64), getattr(got, f).view(np.uint64)), (k, f)


# ---------------------------------------------------------------------------
# exact minimum energy in 1-D (linear program)
# ---------------------------------------------------------------------------
def _lp_1d(hist, alpha0, alpha1, lam):
    """min alpha1 sum_i |u_{i+1} - u_i - v_i| + alpha0 sum_i |v_i - v_{i-1}| + lam sum h|u - c|
    (the discrete Eq. 2 on an N x 1 x 1 block: y/z differences are dropped
    and v_y = v_z = 0 is optimal) as an LP solved by HiGHS."""
    N = hist.shape[0]
    terms = []  # (coefficient dict over u/v, constant, weight)
    for i in range(N - 1):
        terms.append(({("u", i + 1): 1.0, ("u", i): -1.0, ("v", i): -1.0}, 0.0, alpha1))
    for i in range(1, N):
        terms.append(({("v", i): 1.0, ("v", i - 1): -1.0}, 0.0, alpha0))
    for i in range(N):
        for k in range(7):
            if hist[i, k]:
                terms.append(({("u", i): 1.0}, -float(C64[k]), lam * float(hist[i, k])))
    nv = 2 * N + len(terms)
    col = lambda key: key[1] if key[0] == "u" else N + key[1]
    c = np.zeros(nv)
    A, b = [], []
    for t, (coef, const, wt) in enumerate(terms):
        e = 2 * N + t
        c[e] = wt
        for sgn in (1.0, -1.0):
            row = np.zeros(nv)
            for key, val in coef.items():
                row[col(key)] = sgn * val
            row[e] = -1.0
            A.append(row)
            b.append(-sgn * const)
    bounds = [(None, None)] * (2 * N) + [(0, None)] * len(terms)
    res = linprog(c, A_ub=np.array(A), b_ub=np.array(b), bounds=bounds, method="highs")
    assert res.status == 0
    return res.fun, res.x[:N]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_1d_energy_matches_exact_lp(seed):
    rng = np.random.default_rng(10 + seed)
    N = 14
    hist = rand_hist((N, 1, 1), rng, odd=True, lo=1, hi=5)
    a0, a1, lam = oracle.f32(2.0), oracle.f32(1.0), oracle.f32(1.0)
    E_lp, u_lp = _lp_1d(hist, a0, a1, lam)
    st = oracle.solve(hist, (N, 1, 1), C7, 20000)
    P, _ = oracle.primal_energy(hist, (N, 1, 1), C7, st.u, st.v)
    assert P >= E_lp - 1e-9 * max(1.0, E_lp)
    assert P - E_lp <= 1e-8 * max(1.0, E_lp)


# ---------------------------------------------------------------------------
# 3-D: independent smoothed solver, weak duality and the gap
# ---------------------------------------------------------------------------
def _smoothed_minimiser(hist, shape, alpha0, alpha1, lam, eps_list=(1e-2, 1e-4, 1e-6)):
    """Minimise a smoothed Eq. 2 (|.| -> sqrt(.^2 + eps^2)) with L-BFGS and
    continuation in eps; an algorithm unrelated to the primal-dual scheme."""
    nx, ny, nz = shape
    h = torch.tensor(hist[:, :7].astype(np.float64)).reshape(nz, ny, nx, 7)
    c = torch.tensor(C64)

    def fwd(u, ax):  # forward difference along a (z, y, x) axis, 0 on the last slice
        d = torch.diff(u, dim=ax)
        pad = list(u.shape)
        pad[ax] = 1
        return torch.cat([d, torch.zeros(pad, dtype=u.dtype)], dim=ax)

    def bwd(w, ax):  # backward difference, 0 on the first slice
        d = torch.diff(w, dim=ax)
        pad = list(w.shape)
        pad[ax] = 1
        return torch.cat([torch.zeros(pad, dtype=w.dtype), d], dim=ax)

    axes = {0: 2, 1: 1, 2: 0}  # x, y, z -> tensor axis

    def energy(z, eps):
        u = z[: nx * ny * nz].reshape(nz, ny, nx)
        v = z[nx * ny * nz:].reshape(3, nz, ny, nx)
        mask = [torch.ones_like(u) for _ in range(3)]
        for i in range(3):
            m = mask[i]
            idx = [slice(None)] * 3
            idx[axes[i]] = -1
            m[tuple(idx)] = 0
        g = [mask[i] * (fwd(u, axes[i]) - v[i]) for i in range(3)]
        t1 = torch.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2 + eps ** 2).sum()
        D = [[bwd(v[i], axes[j]) for j in range(3)] for i in range(3)]
        E2 = (D[0][0] ** 2 + D[1][1] ** 2 + D[2][2] ** 2
              + 2 * (0.5 * (D[0][1] + D[1][0])) ** 2 + 2 * (0.5 * (D[0][2] + D[2][0])) ** 2
              + 2 * (0.5 * (D[1][2] + D[2][1])) ** 2)
        t0 = torch.sqrt(E2 + eps ** 2).sum()
        td = (h * torch.sqrt((u[..., None] - c) ** 2 + eps ** 2)).sum()
        return alpha1 * t1 + alpha0 * t0 + lam * td

    torch_threads = torch.get_num_threads()
    torch.set_num_threads(1)
    z = np.zeros(4 * nx * ny * nz)
    for eps in eps_list:
        def fg(zz):
            t = torch.tensor(zz, requires_grad=True)
            e = energy(t, eps)
            e.backward()
            return e.item(), t.grad.numpy().copy()
        res = minimize(fg, z, jac=True, method="L-BFGS-B", options=dict(maxiter=4000, maxcor=30, ftol=1e-15,
                                                                         gtol=1e-12))
        z = res.x
    torch.set_num_threads(torch_threads)
    n = nx * ny * nz
    u = z[:n]
    v = z[n:]
    return u, v


@pytest.mark.parametrize("seed", [0])
def test_4cube_cp_beats_independent_smoothed_solver(seed):
    rng = np.random.default_rng(20 + seed)
    shape = (4, 4, 4)
    hist = rand_hist(shape, rng, odd=True, lo=1, hi=6)
    a0, a1, lam = oracle.f32(2.0), oracle.f32(1.0), oracle.f32(1.0)
    st = oracle.solve(hist, shape, C7, 20000)
    P_cp, _ = oracle.primal_energy(hist, shape, C7, st.u, st.v)
    D_cp = oracle.dual_energy(hist, shape, C7, st.u, st.p, st.q)
    u_s, v_s = _smoothed_minimiser(hist, shape, a0, a1, lam)
    P_s, _ = oracle.primal_energy(hist, shape, C7, u_s, v_s)
    # the primal-dual result is at least as good as the independent optimum ...
    assert P_cp <= P_s + 1e-6 * P_s
    assert abs(P_cp - P_s) <= 1e-3 * P_s
    # ... and the dual bound from (p, q) lower-bounds the independent solution
    # (weak duality across two unrelated codes; both solutions lie in the box)
    assert np.abs(u_s).max() <= 1.0 + 1e-6
    assert D_cp <= P_s + 1e-9


@pytest.mark.parametrize("shape,iters", [((4, 4, 4), 20000), ((8, 8, 8), 50000)])
def test_gap_closes_on_fully_observed_blocks(shape, iters):
    rng = np.random.default_rng(7)
    hist = rand_hist(shape, rng, odd=True)
    st = oracle.solve(hist, shape, C7, iters)
    P, D, g = oracle.gap(hist, shape, C7, st)
    assert D <= P + 1e-9
    assert g < 1e-6


def test_weak_duality_random_feasible_points():
    rng = np.random.default_rng(8)
    shape = (5, 4, 3)
    n = 60
    hist = rand_hist(shape, rng, fully=False)
    for _ in range(20):
        u = rng.uniform(-1, 1, n)
        v = rng.normal(size=3 * n)
        v = v.reshape(3, n)
        v = (v / np.maximum(1.0, np.linalg.norm(v, axis=0) / oracle.VBOUND)).ravel()
        p = rng.normal(size=3 * n).reshape(3, n)
        p = (p / np.maximum(1.0, np.linalg.norm(p, axis=0) / 1.0)).ravel()
        q = rng.normal(size=6 * n).reshape(6, n)
        qn = np.sqrt((q[:3] ** 2).sum(0) + 2 * (q[3:] ** 2).sum(0))
        q = (q / np.maximum(1.0, qn / 2.0)).ravel()
        P, _ = oracle.primal_energy(hist, shape, C7, u, v)
        D = oracle.dual_energy(hist, shape, C7, u, p, q)
        assert D <= P + 1e-9


# ---------------------------------------------------------------------------
# zero-level points (Sec. 4.6)
# ---------------------------------------------------------------------------
def test_crossings_of_a_linear_field_lie_on_its_plane():
    nx, ny, nz = 7, 6, 5
    h = 0.5
    origin = np.array([-1.0, 2.0, 0.0], dtype=np.float32)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    # u = 0 on the plane x + 2y - z = 4.25 (voxel units)
    u = (x + 2 * y - z - 4.25).astype(np.float32) / 8
    pts = oracle.crossings(u.ravel(), (nx, ny, nz), origin, h)
    assert len(pts) > 0
    vx = (pts[:, :3] - origin) / h - 0.5  # back to voxel units
    np.testing.assert_allclose(vx[:, 0] + 2 * vx[:, 1] - vx[:, 2], 4.25, atol=1e-5)
    # the number of sign-changing edges, counted independently
    pos = u > 0
    n_edges = ((pos[:, :, 1:] != pos[:, :, :-1]).sum() + (pos[:, 1:, :] != pos[:, :-1, :]).sum()
               + (pos[1:] != pos[:-1]).sum())
    assert len(pts) == n_edges


def test_no_crossings_in_a_constant_sign_field():
    u = np.full(4 * 4 * 4, 0.3, dtype=np.float32)
    assert len(oracle.crossings(u, (4, 4, 4), (0, 0, 0), 1.0)) == 0
    u[21] = 0.0  # voxel (1, 1, 1): u <= 0 counts as inside; its six edges change sign
    pts = oracle.crossings(u, (4, 4, 4), (0, 0, 0), 1.0)
    assert len(pts) == 6 and np.all(pts[:, 3] >= 0)


def test_zero_level_of_the_solved_sphere_is_the_unit_sphere():
    # end to end on the CPU: histograms of 8 noisy ring views of the unit
    # sphere, 300 iterations, crossings; near the cameras' plane (where the
    # data term sees the surface) the points lie on the sphere to a fraction
    # of a voxel (h = 0.094)
    sc = scenes.sphere_scene()
    h, _ = oracle.histograms(sc)
    st = oracle.solve(h, (32, 32, 32), scenes.default_bins(), 300)
    pts = oracle.crossings(st.u.astype(np.float32), (32, 32, 32), sc.grid.origin, sc.grid.h)
    band = np.abs(pts[:, 2]) < 0.5
    r = np.linalg.norm(pts[band, :3], axis=1)
    assert band.sum() > 500
    assert np.median(np.abs(r - 1.0)) < 0.03 and np.percentile(np.abs(r - 1.0), 90) < 0.06


def test_prolongation_takes_the_parent_value():
    rng = np.random.default_rng(12)
    uc = rng.normal(size=4 * 3 * 2)
    uf = oracle.prolongate(uc, (4, 3, 2), (7, 5, 4)).reshape(4, 5, 7)
    Uc = uc.reshape(2, 3, 4)
    for (k, j, i) in [(0, 0, 0), (3, 4, 6), (1, 2, 3), (2, 3, 1)]:
        assert uf[k, j, i] == Uc[k // 2, j // 2, i // 2]


def test_one_level_coarse_to_fine_is_the_plain_solve():
    sc = scenes.sphere_scene(n=12)
    u1 = oracle.coarse_to_fine(sc, 1, 40)
    h, _ = oracle.histograms(sc)
    st = oracle.solve(h, (12, 12, 12), C7, 40)
    np.testing.assert_array_equal(u1, st.u)


# ---------------------------------------------------------------------------
# TV-L1 (Eq. 1)
# ---------------------------------------------------------------------------
def _tvl1_1d_dp(hist, alpha1, lam):
    """Exact minimum of lam sum_i sum_k h_ik |u_i - c_k| + alpha1 sum_i |u_{i+1} - u_i|
    over u in R^N: 1-D TV-L1 with L1 data at the bin centres has a minimiser
    taking values among the centres, so a Viterbi pass over them is exact."""
    N = hist.shape[0]
    c = C64
    cost = lam * np.array([[np.sum(hist[i, :7] * np.abs(v - c)) for v in c] for i in range(N)])
    best = cost[0].copy()
    jump = alpha1 * np.abs(c[:, None] - c[None, :])
    for i in range(1, N):
        best = cost[i] + np.min(best[:, None] + jump, axis=0)
    return float(best.min())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tvl1_1d_energy_matches_exact_dp(seed):
    rng = np.random.default_rng(30 + seed)
    N = 16
    hist = rand_hist((N, 1, 1), rng, odd=False, lo=0, hi=5)
    a1, lam = oracle.f32(1.0), oracle.f32(1.0)
    E = _tvl1_1d_dp(hist, a1, lam)
    st = oracle.solve(hist, (N, 1, 1), C7, 20000, tvl1=True)
    assert not st.v.any() and not st.q.any()
    P, parts = oracle.primal_energy(hist, (N, 1, 1), C7, st.u, st.v)
    assert parts[1] == 0.0
    assert P >= E - 1e-9 * max(1.0, E)
    assert P - E <= 1e-8 * max(1.0, E)


def test_tvl1_gap_closes():
    rng = np.random.default_rng(33)
    shape = (6, 5, 4)
    hist = rand_hist(shape, rng, odd=True)
    st = oracle.solve(hist, shape, C7, 20000, tvl1=True)
    P, D, g = oracle.gap(hist, shape, C7, st, tvl1=True)
    assert D <= P + 1e-9 and g < 1e-6


# ---------------------------------------------------------------------------
# coarse-to-fine levels (Sec. 3.2: coarse-to-fine iterations; Sec. 3.1: the
# band width delta = 6 r scales with the voxel; Sec. 4.5 / Fig. 7: a finer
# part starts from, and freezes its border to, the parent level's indicator)
# ---------------------------------------------------------------------------
def _plane_level_bins(zpi, k, nz_k):
    """Expected rule-0 bin of each coarse z-index of level k for the plane of
    plane_scene(z_plane_index=zpi), worked out by hand: level k has voxel
    edge 2^k h and the same origin, so its centre c sits at (c + 1/2) 2^k h
    and the plane at (zpi + 1/2) h; the offset in the level's own voxels is
    d = (zpi + 1/2) / 2^k - (c + 1/2), and with delta = 3 voxels of that
    level a / delta = d / 3, whose nearest of linspace(-1, 1, 7) is
    floor(d + 3.5) for |d| <= 3 (Alg. 1 clamp, rule 0)."""
    out = []
    for c in range(nz_k):
        d = (zpi + 0.5) / 2 ** k - (c + 0.5)
        assert abs((d % 1.0) - 0.5) > 0.1, "offset on a bin boundary: the case would test rounding"
        assert abs(d) <= 3
        out.append(int(np.floor(d + 3.5)))
    return out


@pytest.mark.parametrize("levels", [2, 3])
def test_coarse_to_fine_levels_follow_the_scaled_plane(levels):
    """Each level of the oracle's coarse-to-fine solve sees the geometry a
    hand computation gives (origin kept, voxel h 2^k, ceil(n / 2^k) voxels,
    delta = 3 h 2^k), its histograms are the plane rule at that scale, its
    solution is the level's own affine indicator (zero TGV energy, the unique
    minimiser), and the finest level returns the plane to 1e-6."""
    zpi = 3.0
    sc = scenes.plane_scene(n=(4, 3, 7), z_plane_index=zpi, n_cams=3)
    rec = []
    u = oracle.coarse_to_fine(sc, levels, 3000, record=rec)
    assert [r["k"] for r in rec] == list(range(levels - 1, -1, -1))
    expect_n = {0: (4, 3, 7), 1: (2, 2, 4), 2: (1, 1, 2)}
    expect_h = {0: 0.25, 1: 0.5, 2: 1.0}
    for r in rec:
        k, g = r["k"], r["grid"]
        assert g.n == expect_n[k] and g.h == expect_h[k]
        np.testing.assert_array_equal(g.origin, sc.grid.origin)
        assert r["delta"] == 0.75 * 2 ** k
        nx, ny, nz = g.n
        H = r["hist"].reshape(nz, ny, nx, 8)
        bins = _plane_level_bins(zpi, k, nz)
        for c, b in enumerate(bins):
            expect = np.zeros(8, dtype=np.uint16)
            expect[b] = 3  # three cameras, vote 1 each
            assert (H[c] == expect).all(), (k, c, H[c, 0, 0], b)
        uk = r["u"].reshape(nz, ny, nx)
        want = np.array([C64[b] for b in bins])
        np.testing.assert_allclose(uk, np.broadcast_to(want[:, None, None], uk.shape), atol=1e-6)
        if k == levels - 1:
            assert not r["u0"].any()  # the coarsest level starts from 0
        else:
            # the start value is the parent level's result, cube by cube
            parent = rec[[q["k"] for q in rec].index(k + 1)]
            pn = parent["grid"].n
            U0 = r["u0"].reshape(nz, ny, nx)
            P = parent["u"].reshape(pn[2], pn[1], pn[0])
            for (z, y, x) in [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz // 2, 0, nx - 1)]:
                assert U0[z, y, x] == P[z // 2, y // 2, x // 2]
    np.testing.assert_allclose(u.reshape(7, 3, 4), np.broadcast_to(C64[[6, 5, 4, 3, 2, 1, 0]][:, None, None],
                                                                   (7, 3, 4)), atol=1e-6)


def test_coarse_to_fine_freezes_only_the_finest_border_to_the_parent():
    """With a 1-voxel halo on the block, the finest level keeps its border at
    the prolongated level-1 solution (known by hand: c_bin of the parent
    cube), while level 1 itself has no frozen layer (it reaches its affine
    indicator up to its faces)."""
    zpi = 3.0
    sc = scenes.plane_scene(n=(4, 3, 7), z_plane_index=zpi, n_cams=3)
    sc.grid = scenes.Grid(sc.grid.origin, sc.grid.h, sc.grid.n, 1)
    rec = []
    u = oracle.coarse_to_fine(sc, 2, 3000, record=rec)
    lvl1, lvl0 = rec
    assert lvl1["grid"].halo == 0 and lvl0["grid"].halo == 1
    parent_bins = _plane_level_bins(zpi, 1, 4)  # [4, 3, 2, 1]
    U = u.reshape(7, 3, 4)
    z, y, x = np.meshgrid(np.arange(7), np.arange(3), np.arange(4), indexing="ij")
    frozen = (x < 1) | (x >= 3) | (y < 1) | (y >= 2) | (z < 1) | (z >= 6)
    want_frozen = np.array([C64[parent_bins[k // 2]] for k in range(7)])[z]
    np.testing.assert_allclose(U[frozen], want_frozen[frozen], atol=1e-6)
    # the border is exactly the start value (never updated)
    np.testing.assert_array_equal(U[frozen], lvl0["u0"].reshape(7, 3, 4)[frozen])


# ---------------------------------------------------------------------------
# energies with a frozen border (Sec. 4.5, Fig. 7: u is fixed on set B, so
# the data term counts free voxels only and the dual pays u.(K^T p) there)
# ---------------------------------------------------------------------------
def _frozen_mask(shape, halo):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = (x < halo) | (x >= nx - halo) | (y < halo) | (y >= ny - halo) | (z < halo) | (z >= nz - halo)
    return m.ravel()


@pytest.mark.parametrize("halo", [1, 2])
def test_weak_duality_with_a_frozen_border(halo):
    """D(p, q) <= P(u, v) for every feasible pair of the problem with u fixed
    on the border: u in [-1, 1] on free voxels, |v| <= 2 sqrt 3, |p| <= a1,
    |q| <= a0 (Frobenius).  Random points, random frozen values."""
    rng = np.random.default_rng(40 + halo)
    shape = (7, 6, 5)
    n = 210
    hist = rand_hist(shape, rng, fully=False)
    for _ in range(30):
        u = rng.uniform(-1, 1, n)
        v = rng.normal(size=(3, n)) * rng.uniform(0.1, 3.0)
        v = (v / np.maximum(1.0, np.linalg.norm(v, axis=0) / oracle.VBOUND)).ravel()
        p = rng.normal(size=(3, n))
        p = (p / np.maximum(1.0, np.linalg.norm(p, axis=0))).ravel()
        q = rng.normal(size=(6, n))
        qn = np.sqrt((q[:3] ** 2).sum(0) + 2 * (q[3:] ** 2).sum(0))
        q = (q / np.maximum(1.0, qn / 2.0)).ravel()
        P, _ = oracle.primal_energy(hist, shape, C7, u, v, halo=halo)
        D = oracle.dual_energy(hist, shape, C7, u, p, q, halo=halo)
        assert D <= P + 1e-9


def test_gap_closes_with_the_border_frozen_at_the_minimiser():
    """Constant histograms (weighted median c_4 = 1/3, odd total) and a 1-voxel
    border frozen at that median: u = 1/3, v = 0 is the minimiser, its energy
    is the data term of the free voxels only (4^3 of them), and the gap
    closes.  A data term counted on frozen voxels would leave P above D by
    the frozen voxels' data."""
    shape = (6, 6, 6)
    n = 216
    hist = np.zeros((n, 8), dtype=np.uint16)
    hist[:, :7] = [1, 0, 2, 0, 3, 1, 0]  # W = 7; sorted: c0 c2 c2 c4 c4 c4 c5 -> median c4
    m = np.float64(C7[4])
    frozen = _frozen_mask(shape, 1)
    assert frozen.sum() == 216 - 64
    st = oracle.solve(hist, shape, C7, 4000, halo=1, u0=np.full(n, m))
    np.testing.assert_allclose(st.u, m, atol=1e-9)
    data_one = sum(int(hist[0, k]) * abs(m - np.float64(C7[k])) for k in range(7))
    P, parts = oracle.primal_energy(hist, shape, C7, st.u, st.v, halo=1)
    assert abs(parts[2] - 64 * data_one) <= 1e-9 * 64 * data_one
    P, D, g = oracle.gap(hist, shape, C7, st, halo=1)
    assert D <= P + 1e-9 and g < 1e-6


@pytest.mark.parametrize("halo", [1, 2])
def test_gap_closes_with_a_random_frozen_border(halo):
    """Random histograms on every voxel and a border frozen at random values
    in [-1, 1]: the minimiser pulls against the border, so p is non-zero
    there and the dual's frozen term u.(K^T p) matters; at convergence the
    primal and dual energies meet (a sign error in that term, or data counted
    on frozen voxels, would keep them apart)."""
    rng = np.random.default_rng(50 + halo)
    shape = (8, 7, 6) if halo == 1 else (9, 8, 8)
    n = int(np.prod(shape))
    hist = rand_hist(shape, rng, odd=True)
    u0 = np.where(_frozen_mask(shape, halo), rng.uniform(-1, 1, n), 0.0)
    st = oracle.solve(hist, shape, C7, 40000, halo=halo, u0=u0)
    frozen = _frozen_mask(shape, halo)
    np.testing.assert_array_equal(st.u[frozen], u0[frozen])
    gu, _ = oracle.apply_KT(st.p, st.q, shape)
    assert np.abs(gu[frozen]).max() > 0.1  # the border term is really exercised
    P, D, g = oracle.gap(hist, shape, C7, st, halo=halo)
    assert D <= P + 1e-9 and g < 1e-6, (P, D, g)
