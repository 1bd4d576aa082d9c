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
    """Cameras in structure-of-arrays form (all float32 / int32): pinhole
    depth maps (model 0) or equirectangular 360-degree scans (model 1)."""

    R: np.ndarray      # [n, 3, 3] float32, world -> camera rotation
    t: np.ndarray      # [n, 3] float32
    intr: np.ndarray   # [n, 4] float32: fx, fy, cx, cy (a scan: fx = pixels per radian)
    wh: np.ndarray     # [n, 2] int32: width, height
    vote: np.ndarray   # [n] int32: vote weight (1, or 5 for LIDAR-like data)
    model: np.ndarray = None  # [n] int32: 0 pinhole, 1 equirectangular scan (None: all pinhole)

    def __post_init__(self):
        if self.model is None:
            self.model = np.zeros(int(self.R.shape[0]), dtype=np.int32)
        self.model = np.asarray(self.model, dtype=np.int32)

    def __len__(self) -> int:
        return int(self.R.shape[0])

    def subset(self, idx: Sequence[int]) -> "Cameras":
        idx = np.asarray(idx, dtype=np.int64)
        return Cameras(self.R[idx].copy(), self.t[idx].copy(), self.intr[idx].copy(),
                       self.wh[idx].copy(), self.vote[idx].copy(), self.model[idx].copy())

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
    import sys
    out = np.zeros(depth64.shape, dtype=np.float32)
    big = depth64.size > (1 << 28)
    for k in range(depth64.shape[0]):
        if big and k % 32 == 0:
            print(f"[scenes] noise {k}/{depth64.shape[0]}", file=sys.stderr, flush=True)
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
    """Camera depth of the heightfield along each pixel ray of pinhole
    camera k (0 where the ray never meets the height range); see
    heightfield_hits."""
    C, d = pixel_rays(cams, k)
    W, H = (int(v) for v in cams.wh[k])
    return heightfield_hits(C, d.reshape(-1, 3), hf, bisect, refine, device).reshape(H, W)


def heightfield_hits(C, dirs: np.ndarray, hf: HeightField, bisect: int = 10, refine: int = 4,
                     device: str = "cpu") -> np.ndarray:
    """Ray parameter s of the first hit C + s d with the heightfield for
    each direction d of dirs [m, 3] (float64; with camera-z component 1, s
    is the camera depth; with unit d, the range).

    Root of g(s) = (C + s d)_Z - H((C + s d)_XY) between the parameters
    where the ray enters and leaves the heightfield's Z range: `bisect`
    bisection steps then `refine` Illinois (modified regula falsi) steps,
    in float64.  Where a ray crosses the surface more than once inside the
    bracket (rare steep spots seen obliquely) the hit may belong to a
    later crossing; 0 where the ray never meets the height range (rays
    that do not descend)."""
    import torch
    dt = torch.from_numpy(np.ascontiguousarray(dirs, dtype=np.float64)).to(device)
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
    return out.cpu().numpy()


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


# ----------------------------------------------------------------------------
# scene 3: synthetic city (boxes on fBm terrain) seen by oblique cameras
# ----------------------------------------------------------------------------
_SCENES_DIR = __import__("os").path.dirname(__import__("os").path.abspath(__file__))
_RAYLIB = __import__("os").path.join(_SCENES_DIR, "libscenes.so")


def build_raycaster() -> str:
    """Compile the heightfield ray caster (input synthesis only) for gfx950."""
    import os
    import subprocess
    src = os.path.join(_SCENES_DIR, "raycast.hip")
    tmp = _RAYLIB + ".tmp"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", tmp, src],
                          stderr=subprocess.DEVNULL)
    os.replace(tmp, _RAYLIB)
    return _RAYLIB


@dataclasses.dataclass
class CityHeightfield:
    """Piecewise-constant heights over the unit square, N x N cells ([j, i])."""

    H: np.ndarray   # [N, N] float32
    zmin: float
    zmax: float
    boxes: np.ndarray  # [n_boxes, 5]: cx, cy, sx, sy, top


def city_heightfield(seed: int = 3, lattice: int = 2048, n_boxes: int = 2000, hurst: float = 0.8,
                     amplitude: float = 0.2) -> CityHeightfield:
    """fBm terrain (peak-to-peak `amplitude`, mid-height 0.5) carrying
    axis-aligned boxes: footprint centres U[0.05, 0.95]^2, sides
    U[0.005, 0.03], heights lognormal (median 0.02, sigma_log 0.6, capped at
    0.2) above the highest terrain point under the footprint."""
    rng = np.random.default_rng(seed)
    z01 = fbm_heightfield(lattice, hurst, seed)
    H = 0.5 + amplitude * (z01 - 0.5)
    N = lattice
    boxes = np.zeros((n_boxes, 5))
    for b in range(n_boxes):
        cx, cy = rng.uniform(0.05, 0.95, size=2)
        sx, sy = rng.uniform(0.005, 0.03, size=2)
        ht = min(0.2, float(np.exp(np.log(0.02) + 0.6 * rng.normal())))
        i0, i1 = int((cx - sx / 2) * N), int(np.ceil((cx + sx / 2) * N))
        j0, j1 = int((cy - sy / 2) * N), int(np.ceil((cy + sy / 2) * N))
        top = float(H[j0:j1, i0:i1].max()) + ht
        H[j0:j1, i0:i1] = np.maximum(H[j0:j1, i0:i1], top)
        boxes[b] = (cx, cy, sx, sy, top)
    H = H.astype(np.float32)
    return CityHeightfield(H, float(H.min()), float(H.max()), boxes)


def city_cameras(n_side: int = 8, headings: int = 4, W: int = 1024, H: int = 1024, f: float = 1024.0,
                 tilt_deg: float = 45.0, standoff: float = 0.5, ground: float = 0.5) -> Cameras:
    """headings x n_side x n_side oblique cameras: each looks at a grid point
    of the ground plane z = `ground` from `standoff` away along its view
    direction's horizontal heading, tilted `tilt_deg` from nadir."""
    Rs, ts = [], []
    tilt = np.deg2rad(tilt_deg)
    for hidx in range(headings):
        th = 2.0 * np.pi * hidx / headings + 0.25 * np.pi
        dirh = np.array([np.cos(th), np.sin(th)])
        for j in range(n_side):
            for i in range(n_side):
                target = np.array([(i + 0.5) / n_side, (j + 0.5) / n_side, ground])
                view = np.array([dirh[0] * np.sin(tilt), dirh[1] * np.sin(tilt), -np.cos(tilt)])
                dist = standoff / np.cos(tilt)
                C = target - dist * view
                R, t = look_at(C, target, [0.0, 0.0, 1.0])
                Rs.append(R)
                ts.append(t)
    return make_cameras(Rs, ts, f, f, W / 2.0, H / 2.0, W, H)


def _cams_f64(cams: Cameras) -> np.ndarray:
    n = len(cams)
    a = np.zeros((n, 16), dtype=np.float64)
    a[:, 0:9] = cams.R.reshape(n, 9).astype(np.float64)
    a[:, 9:12] = cams.t.astype(np.float64)
    a[:, 12:16] = cams.intr.astype(np.float64)
    return np.ascontiguousarray(a)


def render_heightfield_gpu(hf: CityHeightfield, cams: Cameras):
    """Depth maps [n, H, W] float32 of the heightfield on the GPU (torch tensor)."""
    import ctypes
    import os
    import torch
    if not os.path.exists(_RAYLIB):
        raise RuntimeError(f"{_RAYLIB} is not built; run scenes.build_raycaster()")
    L = ctypes.CDLL(_RAYLIB)
    L.scenes_raycast.restype = ctypes.c_int
    L.scenes_raycast.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    Hd = torch.from_numpy(hf.H).cuda()
    W, Hh = (int(v) for v in cams.wh[0])
    out = torch.empty((len(cams), Hh, W), dtype=torch.float32, device="cuda")
    ca = _cams_f64(cams)
    st = torch.cuda.current_stream().cuda_stream
    rc = L.scenes_raycast(Hd.data_ptr(), hf.H.shape[0], hf.zmin, hf.zmax, ca.ctypes.data, len(cams), W, Hh,
                          out.data_ptr(), ctypes.c_void_p(st))
    if rc != 0:
        raise RuntimeError(f"scenes_raycast failed ({rc})")
    return out


def render_heightfield_cpu(hf: CityHeightfield, cams: Cameras) -> np.ndarray:
    """The same cell walk in numpy (vectorised over rays), for small images."""
    N = hf.H.shape[0]
    W, Hh = (int(v) for v in cams.wh[0])
    out = np.zeros((len(cams), Hh, W), dtype=np.float32)
    Hf = hf.H.astype(np.float64)
    for k in range(len(cams)):
        C, d = pixel_rays(cams, k)
        d = d.reshape(-1, 3)
        nr = d.shape[0]
        lo = np.array([0.0, 0.0, hf.zmin])
        hi = np.array([1.0, 1.0, hf.zmax])
        t0 = np.full(nr, 1e-9)
        t1 = np.full(nr, 1e30)
        miss = np.zeros(nr, dtype=bool)
        for a in range(3):
            small = np.abs(d[:, a]) < 1e-300
            miss |= small & ((C[a] < lo[a]) | (C[a] > hi[a]))
            with np.errstate(divide="ignore", invalid="ignore"):
                ta = (lo[a] - C[a]) / d[:, a]
                tb = (hi[a] - C[a]) / d[:, a]
            tmin = np.where(small, -np.inf, np.minimum(ta, tb))
            tmax = np.where(small, np.inf, np.maximum(ta, tb))
            t0 = np.maximum(t0, tmin)
            t1 = np.minimum(t1, tmax)
        alive = ~miss & (t0 < t1)
        x = C[0] + t0 * d[:, 0]
        y = C[1] + t0 * d[:, 1]
        ci = np.clip(np.floor(x * N).astype(np.int64), 0, N - 1)
        cj = np.clip(np.floor(y * N).astype(np.int64), 0, N - 1)
        si = np.where(d[:, 0] > 0, 1, -1)
        sj = np.where(d[:, 1] > 0, 1, -1)
        with np.errstate(divide="ignore", invalid="ignore"):
            tdx = np.where(np.abs(d[:, 0]) > 1e-300, 1.0 / (N * np.abs(d[:, 0])), 1e300)
            tdy = np.where(np.abs(d[:, 1]) > 1e-300, 1.0 / (N * np.abs(d[:, 1])), 1e300)
            tmx = np.where(np.abs(d[:, 0]) > 1e-300, ((ci + (si > 0)) / N - C[0]) / d[:, 0], 1e300)
            tmy = np.where(np.abs(d[:, 1]) > 1e-300, ((cj + (sj > 0)) / N - C[1]) / d[:, 1], 1e300)
        tc = t0.copy()
        res = np.zeros(nr)
        for _ in range(4 * N + 8):
            if not alive.any():
                break
            te = np.minimum(np.minimum(tmx, tmy), t1)
            h = Hf[np.clip(cj, 0, N - 1), np.clip(ci, 0, N - 1)]
            zin = C[2] + tc * d[:, 2]
            zout = C[2] + te * d[:, 2]
            hit = alive & (np.minimum(zin, zout) <= h)
            with np.errstate(divide="ignore", invalid="ignore"):
                th = np.where(zin <= h, tc, (h - C[2]) / d[:, 2])
            res = np.where(hit, th, res)
            alive &= ~hit
            alive &= te < t1
            tc = np.where(alive, te, tc)
            stepx = tmx < tmy
            ci = np.where(alive & stepx, ci + si, ci)
            tmx = np.where(alive & stepx, tmx + tdx, tmx)
            cj = np.where(alive & ~stepx, cj + sj, cj)
            tmy = np.where(alive & ~stepx, tmy + tdy, tmy)
            alive &= (ci >= 0) & (cj >= 0) & (ci < N) & (cj < N)
        out[k] = res.reshape(Hh, W).astype(np.float32)
    return out


def city_scene(seed: int = 3, lattice: int = 2048, n_boxes: int = 2000, W: int = 1024, H: int = 1024,
               f: float = 1024.0, n_side: int = 8, headings: int = 4, sigma: float = 0.3 / 1024,
               outlier_frac: float = 0.01, device: str = "cuda", grid: Grid = None):
    """City depth maps (returned as a Scene with a placeholder grid unless one
    is given) plus the heightfield.  Noise: N(0, sigma^2) on z and uniform
    outliers over the camera-z range of the unit cube."""
    hf = city_heightfield(seed, lattice, n_boxes)
    cams = city_cameras(n_side, headings, W, H, f)
    if device == "cuda":
        clean = render_heightfield_gpu(hf, cams).cpu().numpy().astype(np.float64)
    else:
        clean = render_heightfield_cpu(hf, cams).astype(np.float64)
    g = grid if grid is not None else Grid(np.zeros(3, dtype=np.float32), float(np.float32(1.0 / 256)), (256, 256, 256))
    rng = np.random.default_rng(seed + 7000)
    depth = add_noise(clean, cams, Grid(np.zeros(3, dtype=np.float32), 1.0, (1, 1, 1)), sigma, outlier_frac, rng)
    return Scene(depth, cams, g, name="city"), hf


def city_blocks(scene: Scene, n_blocks: int = 512, e_min: int = 32, e_max: int = 128, halo: int = 2,
                h0: float = 1.0 / 1024, seed: int = 4):
    """Octree-leaf-like blocks on the visible city surface: interior edge
    e = round(exp U[ln e_min, ln e_max]) voxels plus `halo` on each side;
    centres on surface points seen by random cameras; voxel size h0 * 2^m
    with m in 0..3 growing with the distance to the nearest camera (8x range)."""
    rng = np.random.default_rng(seed)
    cams = scene.cams
    Cs = cams.centers()
    blocks = []
    tries = 0
    while len(blocks) < n_blocks and tries < 100 * n_blocks:
        tries += 1
        k = int(rng.integers(len(cams)))
        W, H = (int(v) for v in cams.wh[k])
        px, py = int(rng.integers(W)), int(rng.integers(H))
        z = float(scene.depth[k, py, px])
        if not z > 0:
            continue
        C, d = pixel_rays(cams, k)
        P = C + z * d[py, px]
        dist = float(np.min(np.linalg.norm(Cs - P[None, :], axis=1)))
        e = int(round(np.exp(rng.uniform(np.log(e_min), np.log(e_max)))))
        blocks.append((P, dist, e))
    dists = np.array([b[1] for b in blocks])
    q = np.quantile(dists, [0.25, 0.5, 0.75])
    out = []
    for P, dist, e in blocks:
        m = int(np.searchsorted(q, dist))
        h = float(np.float32(h0 * (2 ** m)))
        n = e + 2 * halo
        origin = (P - 0.5 * n * h).astype(np.float32)
        out.append(Grid(origin, h, (n, n, n), halo))
    return out


# ----------------------------------------------------------------------------
# camera sets
# ----------------------------------------------------------------------------
def concat_cameras(a: Cameras, b: Cameras) -> Cameras:
    return Cameras(np.concatenate([a.R, b.R]), np.concatenate([a.t, b.t]), np.concatenate([a.intr, b.intr]),
                   np.concatenate([a.wh, b.wh]), np.concatenate([a.vote, b.vote]),
                   np.concatenate([a.model, b.model]))


# ----------------------------------------------------------------------------
# 360-degree scans (terrestrial LIDAR, Sec. 3.1) as equirectangular range maps
# ----------------------------------------------------------------------------
def scan360_cameras(centers, W: int = 2048, H: int = 1024, vote: int = 5) -> Cameras:
    """Equirectangular 360-degree scanners at `centers` (world, float64),
    their frames aligned with the world's (R = I, t = -C): column c covers
    azimuths [2 pi c / W, 2 pi (c + 1) / W) from +x towards +y, row r polar
    angles [pi r / H, pi (r + 1) / H) from +z; fx = W / (2 pi) pixels per
    radian; each map holds the range along its pixel rays (model 1)."""
    cs = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    Rs = [np.eye(3) for _ in cs]
    ts = [-c for c in cs]
    cams = make_cameras(Rs, ts, W / (2.0 * math.pi), W / (2.0 * math.pi), 0.0, 0.0, W, H, vote=vote)
    cams.model[:] = 1
    return cams


def scan360_rays(cams: Cameras, k: int):
    """Scanner centre (world, float64) and the unit direction (world) of
    every pixel centre of equirectangular scan k, [H, W, 3]."""
    W, H = (int(v) for v in cams.wh[k])
    phi = 2.0 * math.pi * (np.arange(W, dtype=np.float64) + 0.5) / W
    theta = math.pi * (np.arange(H, dtype=np.float64) + 0.5) / H
    ds = np.empty((H, W, 3), dtype=np.float64)
    ds[..., 0] = np.sin(theta)[:, None] * np.cos(phi)[None, :]
    ds[..., 1] = np.sin(theta)[:, None] * np.sin(phi)[None, :]
    ds[..., 2] = np.cos(theta)[:, None]
    R = cams.R[k].astype(np.float64)
    return cams.centers()[k], ds @ R  # scanner frame -> world: R^T d


def sphere_range(cams: Cameras, k: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Exact range (float64) from scanner k to a sphere along its pixel
    rays (first hit in front of the scanner, also from inside), 0 on a miss."""
    C, d = scan360_rays(cams, k)
    oc = C - np.asarray(center, dtype=np.float64)
    b = d @ oc
    c = float(oc @ oc) - radius * radius
    disc = b * b - c
    hit = disc >= 0
    root = np.sqrt(np.where(hit, disc, 0.0))
    s0, s1 = -b - root, -b + root
    s = np.where(s0 > 0, s0, s1)
    return np.where(hit & (s > 0), s, 0.0)


def terrain_scans360(seed: int = 2, positions=((0.25, 0.25), (0.75, 0.25), (0.25, 0.75), (0.75, 0.75)),
                     height: float = 0.03, W: int = 4096, H: int = 2048, lattice: int = 2048, hurst: float = 0.8,
                     amplitude: float = 0.2, sigma_vox: float = 0.05, n: int = 256, device: str = "cpu"):
    """Terrestrial 360-degree scans of the terrain of terrain_scene (same
    seed, same heightfield) at their own resolution: one equirectangular
    W x H scanner `height` above the ground at each (x, y) position (vote
    5), the range along every pixel ray that descends onto the terrain (0
    elsewhere), N(0, (sigma_vox h)^2) noise on the range and no outliers.
    Returns (range maps [k, H, W] float32, cams)."""
    z01 = fbm_heightfield(lattice, hurst, seed)
    hf = HeightField(z01, base=0.5, amplitude=amplitude)
    centers = [np.array([x, y, float(hf([x], [y])[0]) + height]) for (x, y) in positions]
    cams = scan360_cameras(centers, W, H)
    rng = np.random.default_rng(seed + 3000)
    h = float(np.float32(1.0 / n))
    out = np.zeros((len(cams), H, W), dtype=np.float32)
    for k in range(len(cams)):
        C, d = scan360_rays(cams, k)
        r = heightfield_hits(C, d.reshape(-1, 3), hf, device=device).reshape(H, W)
        valid = r > 0
        r = r + rng.normal(0.0, sigma_vox * h, size=r.shape)
        out[k] = np.where(valid & (r > 0), r, 0.0).astype(np.float32)
    return out, cams


def scan360_sphere_scene(center=(2.2, 0.4, 0.3), W: int = 512, H: int = 256, n: int = 32, extent: float = 1.5,
                         seed: int = 12, sigma: float = 0.001) -> Scene:
    """The unit sphere seen by one equirectangular 360-degree scanner
    (vote 5, low range noise, no outliers) on the block of sphere_scene."""
    cams = scan360_cameras([center], W, H)
    h = np.float32(2.0 * extent / n)
    grid = Grid(np.full(3, -extent, dtype=np.float32), float(h), (n, n, n), 0)
    r = sphere_range(cams, 0)
    rng = np.random.default_rng(seed)
    valid = r > 0
    r = r + rng.normal(0.0, sigma, size=r.shape)
    depth = np.where(valid & (r > 0), r, 0.0).astype(np.float32)[None]
    return Scene(depth, cams, grid, name="scan360-sphere")
