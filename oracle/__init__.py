"""CPU oracle for depth-map fusion by TGV minimisation -- TEST INFRASTRUCTURE.

A plain, slow, obviously correct reference (``oracle.c``: canonical
binary32 pyramids and histogram votes per Algorithm 1; float64 TGV-L1
energy of Eq. 2/3 and its primal-dual minimisation) plus a few closed
forms in numpy.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does,
and this package imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (canonical float flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        c_int, c_long, c_float, c_double = ctypes.c_int, ctypes.c_long, ctypes.c_float, ctypes.c_double
        L.or_pyr_levels.argtypes = [c_int, c_int]
        L.or_pyr_levels.restype = c_int
        L.or_pyr_floats.argtypes = [c_int, c_int]
        L.or_pyr_floats.restype = c_long
        L.or_pyramid.argtypes = [_f32p, c_int, c_int, _f32p]
        L.or_pyramid.restype = None
        L.or_vote_bin.argtypes = [_f32p, c_int, c_int, _f32p, _f32p, _f32p, _f32p, c_float, c_int, c_int, c_int,
                                  c_float, c_float, c_int, c_int, c_int, ctypes.c_void_p]
        L.or_vote_bin.restype = c_int
        L.or_scan_tables.argtypes = [c_int, c_int, _f32p, _f32p, _f32p]
        L.or_scan_tables.restype = None
        L.or_scan_pixel.argtypes = [c_float, c_float, c_float, c_float, c_int, c_int, _f32p, _f32p, _f32p,
                                    ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
        L.or_scan_pixel.restype = None
        L.or_histograms.argtypes = [_f32p, c_int, _f32p, _f32p, _f32p, _i32p, _i32p, _i32p, _f32p, c_float, c_int,
                                    c_int, c_int, c_float, c_float, c_int, c_int, ctypes.c_void_p, c_long, _u16p]
        L.or_histograms.restype = c_long
        L.or_apply_K.argtypes = [c_int, c_int, c_int, _f64p, _f64p, _f64p, _f64p]
        L.or_apply_K.restype = None
        L.or_apply_KT.argtypes = [c_int, c_int, c_int, _f64p, _f64p, _f64p, _f64p]
        L.or_apply_KT.restype = None
        L.or_prox.argtypes = [c_double, _f64p, _f64p, c_int, c_double, c_double]
        L.or_prox.restype = c_double
        L.or_solve.argtypes = [c_int, c_int, c_int, c_int, _u16p, c_int, _f64p, c_double, c_double, c_double,
                               c_double, c_double, c_int, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, c_int]
        L.or_solve.restype = None
        L.or_primal_energy.argtypes = [c_int, c_int, c_int, c_int, _u16p, c_int, _f64p, c_double, c_double, c_double,
                                       _f64p, _f64p, _f64p]
        L.or_primal_energy.restype = c_double
        L.or_dual_energy.argtypes = [c_int, c_int, c_int, c_int, _u16p, c_int, _f64p, c_double, c_double, _f64p,
                                     _f64p, _f64p, c_int]
        L.or_dual_energy.restype = c_double
        L.or_norm_K2.argtypes = [c_int, c_int, c_int, c_int, ctypes.c_uint64]
        L.or_norm_K2.restype = c_double
        L.or_set_threads.argtypes = [c_int]
        L.or_set_threads.restype = None
        L.or_get_threads.argtypes = []
        L.or_get_threads.restype = c_int
        _lib = L
    return _lib


def set_threads(k: int) -> None:
    """Threads of the oracle's per-voxel loops (histogram votes, the dual
    and primal sweeps).  1, the default, is the plain serial oracle; any
    other count gives bit-identical results (each loop writes only its own
    voxel's entries; sums stay serial)."""
    lib().or_set_threads(int(k))


def get_threads() -> int:
    return int(lib().or_get_threads())


class threads:
    """Context manager: run the oracle on k threads inside the block."""

    def __init__(self, k: int):
        self.k = k

    def __enter__(self):
        self.prev = get_threads()
        set_threads(self.k)
        return self

    def __exit__(self, *exc):
        set_threads(self.prev)
        return False


# ----------------------------------------------------------------------------
# pyramids and histograms
# ----------------------------------------------------------------------------
def pyr_levels(W: int, H: int) -> int:
    return int(lib().or_pyr_levels(W, H))


def pyr_floats(W: int, H: int) -> int:
    return int(lib().or_pyr_floats(W, H))


def pyramid(depth: np.ndarray) -> np.ndarray:
    """Pyramid of one depth map [H, W] -> all levels back to back (float32)."""
    d = np.ascontiguousarray(depth, dtype=np.float32)
    H, W = d.shape
    out = np.empty(pyr_floats(W, H), dtype=np.float32)
    lib().or_pyramid(d, W, H, out)
    return out


def pyramid_levels(pyr: np.ndarray, W: int, H: int):
    """Split a packed pyramid into a list of [H_l, W_l] arrays."""
    out, off = [], 0
    w, h = W, H
    while True:
        out.append(pyr[off:off + w * h].reshape(h, w))
        off += w * h
        if w == 1 and h == 1:
            break
        w, h = (w + 1) >> 1, (h + 1) >> 1
    return out


def pyramids(depth: np.ndarray) -> np.ndarray:
    """Pyramids of a stack of depth maps [n, H, W], concatenated."""
    return np.concatenate([pyramid(depth[k]) for k in range(depth.shape[0])])


def bins_params(grid, num_bins=7, rule=0, delta=None, eta_over_delta=3.0):
    """Default binning: delta = 3 h (6 times the voxel radius h/2, Sec. 3.1)."""
    if delta is None:
        delta = float(np.float32(3.0) * np.float32(grid.h))
    return dict(num_bins=int(num_bins), rule=int(rule), delta=float(np.float32(delta)),
                eta_over_delta=float(np.float32(eta_over_delta)))


def histograms(scene, pyr=None, vox=None, num_bins=7, rule=0, delta=None, eta_over_delta=3.0):
    """uint16 [count, 8] histograms of all voxels (vox None) or of the given
    linear voxel indices, and the largest per-voxel vote total."""
    cams, g = scene.cams, scene.grid
    if pyr is None:
        pyr = pyramids(scene.depth)
    bp = bins_params(g, num_bins, rule, delta, eta_over_delta)
    if vox is None:
        count, vptr = g.nvox, None
        vox_arr = None
    else:
        vox_arr = np.ascontiguousarray(vox, dtype=np.int64)
        count, vptr = vox_arr.size, vox_arr.ctypes.data
    out = np.zeros((count, 8), dtype=np.uint16)
    nx, ny, nz = (int(v) for v in g.n)
    mx = lib().or_histograms(np.ascontiguousarray(pyr, dtype=np.float32), len(cams),
                             np.ascontiguousarray(cams.R.reshape(-1), dtype=np.float32),
                             np.ascontiguousarray(cams.t.reshape(-1), dtype=np.float32),
                             np.ascontiguousarray(cams.intr.reshape(-1), dtype=np.float32),
                             np.ascontiguousarray(cams.wh.reshape(-1), dtype=np.int32),
                             np.ascontiguousarray(cams.vote, dtype=np.int32),
                             np.ascontiguousarray(camera_models(cams), dtype=np.int32),
                             np.ascontiguousarray(g.origin, dtype=np.float32), float(g.h), nx, ny, nz,
                             bp["delta"], bp["eta_over_delta"], bp["num_bins"], bp["rule"], vptr, count, out)
    return out, int(mx)


def camera_models(cams) -> np.ndarray:
    """Per-camera model: 0 pinhole depth map, 1 equirectangular 360-degree scan."""
    m = getattr(cams, "model", None)
    return np.zeros(len(cams), dtype=np.int32) if m is None else np.asarray(m, dtype=np.int32)


def scan_tables(W: int, H: int):
    """The column (C, S: W/4 each) and row (K: H) boundary tables of a W x H
    equirectangular scan (float32)."""
    C = np.empty(W // 4, dtype=np.float32)
    S = np.empty(W // 4, dtype=np.float32)
    K = np.empty(H, dtype=np.float32)
    lib().or_scan_tables(W, H, C, S, K)
    return C, S, K


def scan_pixel(x: float, y: float, z: float, rho: float, W: int, H: int, tables=None):
    """(column, row) of a scanner-frame direction in a W x H equirectangular scan."""
    C, S, K = tables if tables is not None else scan_tables(W, H)
    col, row = ctypes.c_int(), ctypes.c_int()
    lib().or_scan_pixel(float(np.float32(x)), float(np.float32(y)), float(np.float32(z)), float(np.float32(rho)),
                        W, H, C, S, K, ctypes.byref(col), ctypes.byref(row))
    return col.value, row.value


def vote_bin(scene, pyr_cam: np.ndarray, cam: int, i: int, j: int, k: int, num_bins=7, rule=0, delta=None,
             eta_over_delta=3.0) -> int:
    cams, g = scene.cams, scene.grid
    bp = bins_params(g, num_bins, rule, delta, eta_over_delta)
    W, H = (int(v) for v in cams.wh[cam])
    model = int(camera_models(cams)[cam])
    tab = None
    if model == 1:
        tab = np.concatenate(scan_tables(W, H))
    return int(lib().or_vote_bin(np.ascontiguousarray(pyr_cam, dtype=np.float32), W, H,
                                 np.ascontiguousarray(cams.R[cam].reshape(-1), dtype=np.float32),
                                 np.ascontiguousarray(cams.t[cam], dtype=np.float32),
                                 np.ascontiguousarray(cams.intr[cam], dtype=np.float32),
                                 np.ascontiguousarray(g.origin, dtype=np.float32), float(g.h), i, j, k,
                                 bp["delta"], bp["eta_over_delta"], bp["num_bins"], bp["rule"], model,
                                 None if tab is None else tab.ctypes.data))


# ----------------------------------------------------------------------------
# solver
# ----------------------------------------------------------------------------
def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def apply_K(u, v, shape):
    nx, ny, nz = shape
    n = nx * ny * nz
    kp = np.zeros(3 * n)
    kq = np.zeros(6 * n)
    lib().or_apply_K(nx, ny, nz, _c64(u).ravel(), _c64(v).ravel(), kp, kq)
    return kp, kq


def apply_KT(p, q, shape):
    nx, ny, nz = shape
    n = nx * ny * nz
    gu = np.zeros(n)
    gv = np.zeros(3 * n)
    lib().or_apply_KT(nx, ny, nz, _c64(p).ravel(), _c64(q).ravel(), gu, gv)
    return gu, gv


def prox(ut, hk, ck, tau, lam):
    hk = _c64(hk)
    ck = _c64(ck)
    return float(lib().or_prox(float(ut), hk, ck, int(hk.size), float(tau), float(lam)))


def norm_K2(shape, iters=200, seed=1):
    nx, ny, nz = shape
    return float(lib().or_norm_K2(nx, ny, nz, iters, seed))


def f32(x) -> float:
    """A parameter as the GPU library sees it (rounded to binary32)."""
    return float(np.float32(x))


class State:
    """Primal-dual state of the oracle: u, v (3), p (3), q (6), ubar, vbar (float64, component-major)."""

    def __init__(self, shape, u0):
        nx, ny, nz = shape
        n = nx * ny * nz
        self.shape = (nx, ny, nz)
        self.u = _c64(u0).ravel().copy()
        self.ubar = self.u.copy()
        self.v = np.zeros(3 * n)
        self.vbar = np.zeros(3 * n)
        self.p = np.zeros(3 * n)
        self.q = np.zeros(6 * n)

    def copy(self):
        s = State.__new__(State)
        s.shape = self.shape
        for k in ("u", "ubar", "v", "vbar", "p", "q"):
            setattr(s, k, getattr(self, k).copy())
        return s


def centers64(centers, num_bins):
    return _c64(np.asarray(centers, dtype=np.float32)[:num_bins].astype(np.float64))


def solve(hist, shape, centers, iters, alpha0=2.0, alpha1=1.0, lam=1.0, tau=None, sigma=None, halo=0,
          num_bins=7, u0=None, state: State = None, tvl1: bool = False) -> State:
    """Run `iters` primal-dual iterations (fresh start from u0, default 0,
    unless a state is given, which is advanced in place and returned).
    Parameters are rounded to binary32 first, as the GPU library takes them."""
    nx, ny, nz = shape
    n = nx * ny * nz
    if tau is None:
        tau = 1.0 / np.sqrt(12.0)
    if sigma is None:
        sigma = tau
    if state is None:
        state = State(shape, np.zeros(n) if u0 is None else u0)
    h = np.ascontiguousarray(hist, dtype=np.uint16).reshape(n, 8)
    lib().or_solve(nx, ny, nz, int(halo), h, int(num_bins), centers64(centers, num_bins), f32(alpha0), f32(alpha1),
                   f32(lam), f32(tau), f32(sigma), int(iters), state.u, state.v, state.p, state.q, state.ubar,
                   state.vbar, int(bool(tvl1)))
    return state


def primal_energy(hist, shape, centers, u, v, alpha0=2.0, alpha1=1.0, lam=1.0, halo=0, num_bins=7):
    nx, ny, nz = shape
    n = nx * ny * nz
    parts = np.zeros(3)
    e = lib().or_primal_energy(nx, ny, nz, int(halo), np.ascontiguousarray(hist, dtype=np.uint16).reshape(n, 8),
                               int(num_bins), centers64(centers, num_bins), f32(alpha0), f32(alpha1), f32(lam),
                               _c64(u).ravel(), _c64(v).ravel(), parts)
    return float(e), parts


VBOUND = 2.0 * np.sqrt(3.0)


def dual_energy(hist, shape, centers, u, p, q, lam=1.0, halo=0, num_bins=7, vbound=VBOUND, tvl1=False):
    nx, ny, nz = shape
    n = nx * ny * nz
    return float(lib().or_dual_energy(nx, ny, nz, int(halo), np.ascontiguousarray(hist, dtype=np.uint16).reshape(n, 8),
                                      int(num_bins), centers64(centers, num_bins), f32(lam), float(vbound),
                                      _c64(u).ravel(), _c64(p).ravel(), _c64(q).ravel(), int(bool(tvl1))))


def gap(hist, shape, centers, st: State, alpha0=2.0, alpha1=1.0, lam=1.0, halo=0, num_bins=7, tvl1=False):
    """(P, D, relative gap (P - D) / max(P, 1))."""
    P, _ = primal_energy(hist, shape, centers, st.u, st.v, alpha0, alpha1, lam, halo, num_bins)
    D = dual_energy(hist, shape, centers, st.u, st.p, st.q, lam, halo, num_bins, tvl1=tvl1)
    return P, D, (P - D) / max(P, 1.0)


# ----------------------------------------------------------------------------
# closed forms (numpy)
# ----------------------------------------------------------------------------
def weighted_median_interval(hk, ck):
    """Minimisers [lo, hi] of sum_k h_k |w - c_k| (the weighted median); for
    an odd total weight lo == hi.  Empty histograms give (-inf, inf)."""
    hk = np.asarray(hk, dtype=np.int64)
    ck = np.asarray(ck, dtype=np.float64)
    W = int(hk.sum())
    if W == 0:
        return -np.inf, np.inf
    expanded = np.repeat(ck, hk)  # sorted because centres ascend
    if W % 2 == 1:
        m = float(expanded[W // 2])
        return m, m
    return float(expanded[W // 2 - 1]), float(expanded[W // 2])


# ----------------------------------------------------------------------------
# zero level (Sec. 4.6)
# ----------------------------------------------------------------------------
def crossings(u, shape, origin, h) -> np.ndarray:
    """Iso-surface points of u = 0: on every grid edge (x, x + e_i) whose end
    values have different signs (u > 0 against u <= 0), the point
    origin + (x + 1/2 + t e_i) h with t = u(x) / (u(x) - u(x + e_i)).
    Binary32 arithmetic in the order written; rows (X, Y, Z, i) in voxel
    order, then axis order."""
    nx, ny, nz = shape
    f = np.float32
    U = np.asarray(u, dtype=np.float32).reshape(nz, ny, nx)
    o = np.asarray(origin, dtype=np.float32)
    h = f(h)
    rows = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                a = U[z, y, x]
                c = [o[0] + (f(x) + f(0.5)) * h, o[1] + (f(y) + f(0.5)) * h, o[2] + (f(z) + f(0.5)) * h]
                nb = [(x + 1 < nx, (z, y, x + 1)), (y + 1 < ny, (z, y + 1, x)), (z + 1 < nz, (z + 1, y, x))]
                for i, (ok, j) in enumerate(nb):
                    if not ok:
                        continue
                    b = U[j]
                    if (a > 0) != (b > 0):
                        t = f(a / f(a - b))
                        p = list(c)
                        p[i] = f(c[i] + f(t * h))
                        rows.append([p[0], p[1], p[2], f(i)])
    return np.array(rows, dtype=np.float32).reshape(-1, 4)


# ----------------------------------------------------------------------------
# coarse-to-fine (Sec. 3.2, Sec. 4.5)
# ----------------------------------------------------------------------------
class _Grid:
    def __init__(self, origin, h, n, halo=0):
        self.origin = np.asarray(origin, dtype=np.float32)
        self.h = float(np.float32(h))
        self.n = tuple(int(v) for v in n)
        self.halo = int(halo)

    @property
    def nvox(self):
        return self.n[0] * self.n[1] * self.n[2]


class _Scene:
    def __init__(self, depth, cams, grid):
        self.depth, self.cams, self.grid = depth, cams, grid


def prolongate(u_coarse, coarse_shape, fine_shape) -> np.ndarray:
    """Each fine voxel takes the value of its parent cube: u_f(i, j, k) =
    u_c(i // 2, j // 2, k // 2) (the paper freezes a part's border to the
    parent level's indicator and refines from it)."""
    cx, cy, cz = coarse_shape
    fx, fy, fz = fine_shape
    U = np.asarray(u_coarse).reshape(cz, cy, cx)
    k, j, i = np.meshgrid(np.arange(fz) // 2, np.arange(fy) // 2, np.arange(fx) // 2, indexing="ij")
    return U[k, j, i].ravel()


def coarse_to_fine(scene, levels, iters, alpha0=2.0, alpha1=1.0, lam=1.0, tau=None, sigma=None, num_bins=7,
                   rule=0, centers=None, record=None):
    """Solve the block on levels-1 .. 0 with voxel size h 2^k (ceil(n / 2^k)
    voxels per axis, same origin, delta scaled with the voxel): each level's
    histograms come from the depth maps, its start value is the prolongated
    coarser solution (0 on the coarsest) and its border layer (the finest
    level's halo; none on coarser levels) stays frozen.  When `record` is a
    list, one dict per level (coarsest first) is appended to it: the level
    k, its grid, delta, histograms, start value u0 and result u."""
    g0 = scene.grid
    grids = [_Grid(g0.origin, g0.h, g0.n, g0.halo)]
    for k in range(1, levels):
        p = grids[-1]
        grids.append(_Grid(p.origin, np.float32(p.h) * np.float32(2.0), tuple((v + 1) // 2 for v in p.n), 0))
    delta0 = np.float32(3.0) * np.float32(g0.h)
    if centers is None:
        centers = np.full(8, np.inf, dtype=np.float32)
        centers[:num_bins] = np.linspace(-1.0, 1.0, num_bins).astype(np.float32)
    pyr = pyramids(scene.depth)
    u = None
    for k in range(levels - 1, -1, -1):
        gk = grids[k]
        hk, _ = histograms(_Scene(scene.depth, scene.cams, gk), pyr, num_bins=num_bins, rule=rule,
                           delta=float(delta0 * np.float32(2 ** k)))
        u0 = np.zeros(gk.nvox) if u is None else prolongate(u, grids[k + 1].n, gk.n)
        st = solve(hk, gk.n, centers, iters, alpha0, alpha1, lam, tau, sigma, halo=gk.halo, num_bins=num_bins, u0=u0)
        u = st.u
        if record is not None:
            record.append(dict(k=k, grid=gk, delta=float(delta0 * np.float32(2 ** k)), hist=hk, u0=u0, u=u.copy()))
    return u
