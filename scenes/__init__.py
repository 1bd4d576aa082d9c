"""Seeded synthetic scenes: depth maps, pinhole cameras and voxel blocks.

This module produces the *inputs* of depth-map fusion and nothing else: it
holds none of the fusion arithmetic (no pyramids, no histogram rule, no
solver).  Both the HIP path and the CPU oracle consume what it returns.

Camera convention (shared by every consumer of these arrays):
  * world -> camera: Xc = R @ X + t, R row-major 3x3 (float32);
  * camera frame: x right, y down (image rows grow downwards), z forward;
  * a pixel column i covers [i, i+1), so its centre is i + 0.5;
  * projection: px = fx * Xc/Zc + cx, py = fy * Yc/Zc + cy;
  * a depth map stores the camera-frame z of the first surface hit along
    the ray through the pixel centre; 0 marks "no sample" (background).

Noise model (the paper's inputs are noisy stereo depth maps, Sec. 3.1):
Gaussian noise N(0, sigma^2) on z, then a uniformly chosen fraction of the
valid pixels is replaced by outliers drawn uniformly from the camera-z
range of the block's eight corners.

Every random draw goes through ``numpy.random.default_rng(seed)`` (PCG64)
on the host, so a seed fixes every array bit for bit.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence

import numpy as np


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Cameras:
    """Pinhole cameras in structure-of-arrays form (all float32 / int32)."""

    R: np.ndarray      # [n, 3, 3] float32, world -> camera rotation
    t: np.ndarray      # [n, 3] float32
    intr: np.ndarray   # [n, 4] float32: fx, fy, cx, cy
    wh: np.ndarray     # [n, 2] int32: width, height
    vote: np.ndarray   # [n] int32: vote weight (1, or 5 for LIDAR-like data)

    def __len__(self) -> int:
        return int(self.R.shape[0])

    def subset(self, idx: Sequence[int]) -> "Cameras":
        idx = np.asarray(idx, dtype=np.int64)
        return Cameras(self.R[idx].copy(), self.t[idx].copy(), self.intr[idx].copy(),
                       self.wh[idx].copy(), self.vote[idx].copy())

    def centers(self) -> np.ndarray:
        """Camera centres in world coordinates, float64: C = -R^T t."""
        R = self.R.astype(np.float64)
        t = self.t.astype(np.float64)
        return -np.einsum("nji,nj->ni", R, t)


@dataclasses.dataclass
class Grid:
    """A regular voxel block: voxel (i, j, k) has centre origin + (idx + 0.5) * h."""

    origin: np.ndarray  # [3] float32, corner of the padded grid
    h: float            # voxel edge (representable in float32)
    n: tuple            # (nx, ny, nz)
    halo: int = 0       # cells closer than `halo` to a face keep u frozen

    @property
    def nvox(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def corners(self) -> np.ndarray:
        o = self.origin.astype(np.float64)
        ext = np.array(self.n, dtype=np.float64) * float(self.h)
        out = []
        for c in range(8):
            out.append(o + ext * np.array([(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1], dtype=np.float64))
        return np.stack(out)


@dataclasses.dataclass
class Scene:
    depth: np.ndarray   # [n_cams, H, W] float32 (0 = invalid)
    cams: Cameras
    grid: Grid
    name: str = ""

    def digest(self) -> str:
        hsh = hashlib.sha256()
        for a in (self.depth, self.cams.R, self.cams.t, self.cams.intr, self.cams.wh, self.cams.vote,
                  self.grid.origin):
            hsh.update(np.ascontiguousarray(a).tobytes())
        hsh.update(repr((float(self.grid.h), tuple(int(x) for x in self.grid.n), int(self.grid.halo))).encode())
        return hsh.hexdigest()


# ----------------------------------------------------------------------------
# camera helpers
# ----------------------------------------------------------------------------
def look_at(center, target, up) -> tuple:
    """World->camera rotation and translation (float64) for a camera at
    `center` looking at `target`; image y points away from `up`."""
    c = np.asarray(center, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ c
    return R, t


def make_cameras(Rs, ts, fx, fy, cx, cy, W, H, vote=1) -> Cameras:
    n = len(Rs)
    R = np.asarray(Rs, dtype=np.float64).astype(np.float32).reshape(n, 3, 3)
    t = np.asarray(ts, dtype=np.float64).astype(np.float32).reshape(n, 3)
    intr = np.tile(np.array([fx, fy, cx, cy], dtype=np.float32), (n, 1))
    wh = np.tile(np.array([W, H], dtype=np.int32), (n, 1))
    votes = np.full(n, vote, dtype=np.int32)
    return Cameras(R, t, intr, wh, votes)


def pixel_rays(cams: Cameras, k: int):
    """Ray origin (world, float64) and per-pixel directions d with camera-z
    component 1, so that the hit point is C + z * d for camera depth z."""
    R = cams.R[k].astype(np.float64)
    fx, fy, cx, cy = (float(v) for v in cams.intr[k])
    W, H = (int(v) for v in cams.wh[k])
    xs = (np.arange(W, dtype=np.float64) + 0.5 - cx) / fx
    ys = (np.arange(H, dtype=np.float64) + 0.5 - cy) / fy
    dc = np.empty((H, W, 3), dtype=np.float64)
    dc[..., 0] = xs[None, :]
    dc[..., 1] = ys[:, None]
    dc[..., 2] = 1.0
    dw = dc @ R  # row vectors: (R^T d)^T = d^T R
    return cams.centers()[k], dw


# ----------------------------------------------------------------------------
# noise
# ----------------------------------------------------------------------------
def camera_z_range(cams: Cameras, k: int, grid: Grid) -> tuple:
    R = cams.R[k].astype(np.float64)
    t = cams.t[k].astype(np.float64)
    z = grid.corners() @ R[2] + t[2]
    lo = max(float(z.min()), 1e-3)
    hi = max(float(z.max()), lo * (1 + 1e-3))
    return lo, hi


def add_noise(depth64: np.ndarray, cams: Cameras, grid: Grid, sigma: float, outlier_frac: float,
              rng: np.random.Generator) -> np.ndarray:
    """Gaussian z-noise then uniform outliers on valid pixels; returns float32 maps."""
    out = np.zeros(depth64.shape, dtype=np.float32)
    for k in range(depth64.shape[0]):
        d = depth64[k].copy()
        valid = d > 0
        if sigma > 0:
            d = d + rng.normal(0.0, sigma, size=d.shape)
        nvalid = int(valid.sum())
        n_out = int(round(outlier_frac * nvalid))
        if n_out > 0:
            flat = np.flatnonzero(valid.ravel())
            pick = rng.choice(flat, size=n_out, replace=False)
            lo, hi = camera_z_range(cams, k, grid)
            d.ravel()[pick] = rng.uniform(lo, hi, size=n_out)
        d = np.where(valid & (d > 0), d, 0.0)
        out[k] = d.astype(np.float32)
    return out


# ----------------------------------------------------------------------------
# scene 1: unit sphere seen from a ring of cameras
# ----------------------------------------------------------------------------
def sphere_depth(cams: Cameras, k: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Exact ray/sphere camera depth (float64), 0 where the ray misses."""
    C, d = pixel_rays(cams, k)
    oc = C - np.asarray(center, dtype=np.float64)
    a = np.einsum("hwc,hwc->hw", d, d)
    b = d @ oc
    c = float(oc @ oc) - radius * radius
    disc = b * b - a * c
    hit = disc >= 0
    s = np.where(hit, (-b - np.sqrt(np.where(hit, disc, 0.0))) / a, 0.0)
    return np.where(hit & (s > 0), s, 0.0)


def sphere_scene(seed: int = 1, n_cams: int = 8, W: int = 128, H: int = 128, f: float = 128.0,
                 ring_radius: float = 3.0, sigma: float = 0.005, outlier_frac: float = 0.02,
                 n: int = 32, extent: float = 1.5) -> Scene:
    """Unit sphere at the origin; cameras on a ring in the z=0 plane looking
    at the origin with +z up; the block spans [-extent, extent]^3."""
    Rs, ts = [], []
    for k in range(n_cams):
        ang = 2.0 * math.pi * k / n_cams
        C = ring_radius * np.array([math.cos(ang), math.sin(ang), 0.0])
        R, t = look_at(C, [0.0, 0.0, 0.0], [0.0, 0.0, 1.0])
        Rs.append(R)
        ts.append(t)
    cams = make_cameras(Rs, ts, f, f, W / 2.0, H / 2.0, W, H)
    h = np.float32(2.0 * extent / n)
    grid = Grid(np.full(3, -extent, dtype=np.float32), float(h), (n, n, n), 0)
    clean = np.stack([sphere_depth(cams, k) for k in range(n_cams)])
    rng = np.random.default_rng(seed)
    depth = add_noise(clean, cams, grid, sigma, outlier_frac, rng)
    return Scene(depth, cams, grid, name=f"sphere{n}")


# ----------------------------------------------------------------------------
# scene 2: fBm heightfield terrain seen by nadir cameras
# ----------------------------------------------------------------------------
def fbm_heightfield(size: int, hurst: float, seed: int) -> np.ndarray:
    """Periodic fractional-Brownian-motion surface by spectral synthesis:
    power spectrum proportional to |k|^-(2H+2); normalised to [0, 1]."""
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(size)[None, :]
    ky = np.fft.fftfreq(size)[:, None]
    kk = np.sqrt(kx * kx + ky * ky)
    kk[0, 0] = 1.0
    amp = kk ** (-(2.0 * hurst + 2.0) / 2.0)
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(size, size))
    mag = rng.normal(size=(size, size))
    spec = amp * mag * np.exp(1j * phase)
    z = np.real(np.fft.ifft2(spec))
    z -= z.min()
    z /= z.max()
    return z


class HeightField:
    """Bilinear, periodic heightfield over the unit square [0,1)^2 (float64).
    Lookups run in torch so that large ray batches use every host core."""

    def __init__(self, z01: np.ndarray, base: float, amplitude: float):
        self.z = base + amplitude * (np.asarray(z01, dtype=np.float64) - 0.5)
        self.n = self.z.shape[0]
        self.zmin = float(self.z.min())
        self.zmax = float(self.z.max())
        self._zt = {}

    def table(self, device):
        import torch
        key = str(device)
        if key not in self._zt:
            self._zt[key] = torch.from_numpy(self.z.ravel()).to(device)
        return self._zt[key]

    def lookup(self, x, y):
        """x, y: torch float64 tensors (world units); returns heights."""
        import torch
        n = self.n
        z = self.table(x.device)
        gx = x * n - 0.5
        gy = y * n - 0.5
        x0 = torch.floor(gx)
        y0 = torch.floor(gy)
        fx = gx - x0
        fy = gy - y0
        i0 = torch.remainder(x0.to(torch.int64), n)
        j0 = torch.remainder(y0.to(torch.int64), n)
        i1 = torch.remainder(i0 + 1, n)
        j1 = torch.remainder(j0 + 1, n)
        z00 = z[j0 * n + i0]
        z01 = z[j0 * n + i1]
        z10 = z[j1 * n + i0]
        z11 = z[j1 * n + i1]
        return (z00 * (1 - fx) + z01 * fx) * (1 - fy) + (z10 * (1 - fx) + z11 * fx) * fy

    def __call__(self, x, y):
        import torch
        xt = torch.as_tensor(np.asarray(x, dtype=np.float64))
        yt = torch.as_tensor(np.asarray(y, dtype=np.float64))
        return self.lookup(xt, yt).numpy()


def heightfield_depth(cams: Cameras, k: int, hf: HeightField, bisect: int = 10, refine: int = 4,
                      device: str = "cpu") -> np.ndarray:
    """Camera depth of the heightfield along each pixel ray.

    Root of g(z) = (C + z d)_Z - H((C + z d)_XY) between the depths where
    the ray enters and leaves the heightfield's Z range: `bisect` bisection
    steps then `refine` Illinois (modified regula falsi) steps, in float64.
    Where a ray crosses the surface more than once inside the bracket (rare
    steep spots seen obliquely) the depth may belong to a later crossing;
    0 where the ray never meets the height range."""
    import torch
    C, d = pixel_rays(cams, k)
    dt = torch.from_numpy(d.reshape(-1, 3)).to(device)
    Cx, Cy, Cz = (float(c) for c in C)
    dz = dt[:, 2]
    ok = dz < 0
    safe = torch.where(ok, dz, torch.full_like(dz, -1.0))
    lo = torch.clamp((hf.zmax - Cz) / safe, min=1e-9)
    hi = (hf.zmin - Cz) / safe
    ok &= hi > lo

    def g(zz):
        return (Cz + zz * dt[:, 2]) - hf.lookup(Cx + zz * dt[:, 0], Cy + zz * dt[:, 1])

    glo = g(lo)
    ghi = g(hi)
    ok &= (glo >= 0) & (ghi <= 0)
    for _ in range(bisect):
        mid = 0.5 * (lo + hi)
        gm = g(mid)
        above = gm > 0
        lo = torch.where(above, mid, lo)
        glo = torch.where(above, gm, glo)
        hi = torch.where(above, hi, mid)
        ghi = torch.where(above, ghi, gm)
    side = torch.zeros_like(lo)
    for _ in range(refine):
        den = glo - ghi
        den = torch.where(den > 0, den, torch.ones_like(den))
        zm = lo + (hi - lo) * (glo / den)
        zm = torch.minimum(torch.maximum(zm, lo), hi)
        gm = g(zm)
        above = gm > 0
        # Illinois: halve the retained end's value when the same side repeats
        glo_new = torch.where(above, gm, torch.where(side < 0, glo * 0.5, glo))
        ghi_new = torch.where(above, torch.where(side > 0, ghi * 0.5, ghi), gm)
        lo = torch.where(above, zm, lo)
        hi = torch.where(above, hi, zm)
        glo, ghi = glo_new, ghi_new
        side = torch.where(above, torch.ones_like(side), -torch.ones_like(side))
    zc = torch.where(glo - ghi > 0, lo + (hi - lo) * (glo / torch.where(glo - ghi > 0, glo - ghi, torch.ones_like(glo))), 0.5 * (lo + hi))
    out = torch.where(ok, zc, torch.zeros_like(zc))
    W, H = (int(v) for v in cams.wh[k])
    return out.reshape(H, W).cpu().numpy()


def terrain_scene(seed: int = 2, n: int = 256, n_side: int = 8, W: int = 1024, H: int = 1024,
                  f: float = 1536.0, altitude: float = 1.5, lattice: int = 2048, hurst: float = 0.8,
                  amplitude: float = 0.2, sigma_vox: float = 0.3, outlier_frac: float = 0.01,
                  origin=(0.0, 0.0, 0.0), extent: float = 1.0, device: str = "cpu") -> Scene:
    """fBm terrain (peak-to-peak `amplitude`, centred at mid-height of the
    unit cube) under an n_side x n_side grid of nadir cameras at `altitude`
    above mid-height; the block is n^3 voxels over [0, extent]^3 + origin."""
    z01 = fbm_heightfield(lattice, hurst, seed)
    hf = HeightField(z01, base=0.5, amplitude=amplitude)
    Rs, ts = [], []
    for jy in range(n_side):
        for ix in range(n_side):
            C = np.array([(ix + 0.5) / n_side, (jy + 0.5) / n_side, 0.5 + altitude])
            R = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, -1.0]])
            Rs.append(R)
            ts.append(-R @ C)
    cams = make_cameras(Rs, ts, f, f, W / 2.0, H / 2.0, W, H)
    h = float(np.float32(extent / n))
    grid = Grid(np.asarray(origin, dtype=np.float32), h, (n, n, n), 0)
    clean = np.stack([heightfield_depth(cams, k, hf, device=device) for k in range(len(cams))])
    rng = np.random.default_rng(seed + 1000)
    depth = add_noise(clean, cams, grid, sigma_vox * h, outlier_frac, rng)
    return Scene(depth, cams, grid, name=f"terrain{n}")


# ----------------------------------------------------------------------------
# simple analytic scenes used by the pins
# ----------------------------------------------------------------------------
def plane_scene(n=(7, 5, 4), z_plane_index: float = 3.0, n_cams: int = 1, W: int = 64, H: int = 64,
                f: float = 64.0, distance: float = 20.0, h: float = 0.25, vote: int = 1) -> Scene:
    """Fronto-parallel plane Z = z0 seen by cameras looking along +Z.

    The block's voxel centres along Z are origin_z + (k + 0.5) h; the plane
    sits on the centre plane k = z_plane_index.  The cameras sit on the -Z
    side at camera depth `distance` from the plane; every pixel sees the
    plane, so the depth map is the constant `distance` (exact in float32)
    and every pyramid level equals it.  Several cameras are shifted
    sideways (pure translation keeps the depth constant)."""
    nx, ny, nz = n
    origin = np.array([-nx * h / 2.0, -ny * h / 2.0, 0.0], dtype=np.float32)
    z0 = float(origin[2]) + (z_plane_index + 0.5) * h
    R = np.eye(3)
    Rs, ts = [], []
    for k in range(n_cams):
        C = np.array([0.01 * k * h, -0.013 * k * h, z0 - distance])
        Rs.append(R)
        ts.append(-R @ C)
    cams = make_cameras(Rs, ts, f, f, W / 2.0, H / 2.0, W, H, vote=vote)
    grid = Grid(origin, float(np.float32(h)), tuple(int(v) for v in n), 0)
    depth = np.full((n_cams, H, W), np.float32(distance), dtype=np.float32)
    return Scene(depth, cams, grid, name="plane")


def default_bins(num_bins: int = 7, rule: int = 0):
    """Bin centres (float32) for the two assignment rules: rule 0 puts
    num_bins centres uniformly on [-1, 1] (ends included); rule 1 uses the
    midpoints of num_bins equal cells of [-1, 1]."""
    if rule == 0:
        c = np.linspace(-1.0, 1.0, num_bins)
    else:
        c = -1.0 + (2.0 * np.arange(num_bins) + 1.0) / num_bins
    out = np.full(8, np.inf, dtype=np.float32)
    out[:num_bins] = c.astype(np.float32)
    return out


def config_scene(k: int, **kw) -> Scene:
    """Scene of one of the named workloads (1 = sphere 32^3, 2 = terrain 256^3)."""
    if k == 1:
        return sphere_scene(**kw)
    if k == 2:
        return terrain_scene(**kw)
    raise ValueError(f"no scene for workload {k}")
