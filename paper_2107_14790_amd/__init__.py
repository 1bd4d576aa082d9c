"""Python binding of libtgv (MI355X / gfx950 HIP library for depth-map fusion
by TGV minimisation).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/tgv.h.  Torch tensors carry
device memory and torch's current stream carries the ordering.  There is no
CPU fallback: importing this package without the built library, or calling
it without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtgv.so")

TGV_OK, TGV_E_INVAL, TGV_E_NOMEM, TGV_E_DEVICE, TGV_E_OVERFLOW, TGV_E_UNSUPPORTED = range(6)
STORE_F32, STORE_F16, STORE_BF16 = 0, 1, 2
SCHED_FUSED, SCHED_SPLIT, SCHED_FUSED_REF, SCHED_FUSED2, SCHED_AUTO = 0, 1, 2, 3, 4
FLAG_GRAPH = 1
FLAG_TVL1 = 2
FLAG_LEAVE_OPEN = 4
NOALLOC_MAX_BYTES = 64 << 20  # TGV_NOALLOC_MAX_BYTES
MODEL_PINHOLE, MODEL_SCAN360 = 0, 1
HIST_ACCUMULATE = 1
STORAGE_NAMES = {"f32": STORE_F32, "f16": STORE_F16, "bf16": STORE_BF16}


class TgvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libtgv status {status}: {msg}")
        self.status = status


# ---------------------------------------------------------------------------
# ABI structs (must match include/tgv.h)
# ---------------------------------------------------------------------------
class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("vote", ctypes.c_int32),
                ("model", ctypes.c_int32)]


class GridT(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("h", ctypes.c_float), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("halo", ctypes.c_int32)]


class BinsT(ctypes.Structure):
    _fields_ = [("num_bins", ctypes.c_int32), ("rule", ctypes.c_int32), ("centers", ctypes.c_float * 8),
                ("delta", ctypes.c_float), ("eta_over_delta", ctypes.c_float)]


class ParamsT(ctypes.Structure):
    _fields_ = [("alpha0", ctypes.c_float), ("alpha1", ctypes.c_float), ("lam", ctypes.c_float),
                ("tau", ctypes.c_float), ("sigma", ctypes.c_float), ("iters", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("schedule", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("tile_z", ctypes.c_int32), ("flags", ctypes.c_int32)]


class StatsT(ctypes.Structure):
    _fields_ = [("primal", ctypes.c_double), ("dual", ctypes.c_double), ("gap_rel", ctypes.c_double),
                ("parts", ctypes.c_double * 3), ("nonfinite", ctypes.c_int64), ("iters_done", ctypes.c_int64)]


assert ctypes.sizeof(Camera) == 80 and ctypes.sizeof(GridT) == 32 and ctypes.sizeof(BinsT) == 48
assert ctypes.sizeof(ParamsT) == 44 and ctypes.sizeof(StatsT) == 64

_vp = ctypes.c_void_p
_SIGS = {
    "tgv_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "tgv_destroy": (None, [_vp]),
    "tgv_last_error": (ctypes.c_char_p, [_vp]),
    "tgv_pyramid_levels": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
    "tgv_pyramid_floats": (ctypes.c_int64, [ctypes.c_int32, ctypes.c_int32]),
    "tgv_build_pyramids": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp]),
    "tgv_cull_cameras": (ctypes.c_int32, [ctypes.POINTER(Camera), ctypes.c_int32, ctypes.POINTER(GridT),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "tgv_build_histograms": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Camera),
                                            ctypes.c_int32, ctypes.POINTER(GridT), ctypes.POINTER(BinsT), _vp, _vp]),
    "tgv_build_histograms_ex": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Camera),
                                               ctypes.c_int32, ctypes.POINTER(GridT), ctypes.POINTER(BinsT),
                                               ctypes.c_int32, ctypes.c_int32, _vp, _vp]),
    "tgv_state_create": (ctypes.c_int, [_vp, ctypes.POINTER(GridT), ctypes.c_int32, ctypes.POINTER(_vp)]),
    "tgv_state_destroy": (None, [_vp]),
    "tgv_state_wrap": (ctypes.c_int, [_vp, ctypes.POINTER(GridT), ctypes.c_int32, _vp, ctypes.c_int64,
                                      ctypes.POINTER(_vp)]),
    "tgv_state_bytes": (ctypes.c_int64, [ctypes.POINTER(GridT), ctypes.c_int32]),
    "tgv_state_reset": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "tgv_state_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tgv_state_import": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "tgv_solve": (ctypes.c_int, [_vp, ctypes.POINTER(GridT), _vp, ctypes.POINTER(BinsT), ctypes.POINTER(ParamsT),
                                 _vp, _vp, ctypes.POINTER(StatsT), _vp]),
    "tgv_solve_noalloc": (ctypes.c_int, [_vp, ctypes.POINTER(GridT), _vp, ctypes.POINTER(BinsT),
                                         ctypes.POINTER(ParamsT), _vp, _vp]),
    "tgv_energy": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(BinsT), ctypes.POINTER(ParamsT),
                                  ctypes.POINTER(StatsT), _vp]),
    "tgv_extract_crossings": (ctypes.c_int, [_vp, ctypes.POINTER(GridT), _vp, _vp, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64), _vp]),
    "tgv_stream_copy": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp]),
    "tgv_prolongate": (ctypes.c_int, [_vp, ctypes.POINTER(GridT), _vp, ctypes.POINTER(GridT), _vp, _vp]),
    "tgv_solve_coarse_to_fine": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Camera),
                                                ctypes.c_int32, ctypes.POINTER(GridT), ctypes.POINTER(BinsT),
                                                ctypes.POINTER(ParamsT), ctypes.c_int32, _vp, _vp]),
    "tgv_solve_batch": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                       ctypes.POINTER(BinsT), ctypes.POINTER(ParamsT), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(StatsT), _vp]),
}
EXPORTED = tuple(_SIGS)

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtgv.so and declare every exported entry point (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtgv.so not built at {path}; run __graft_entry__.build() or "
                          f"python paper_2107_14790_amd/build.py")
    L = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libtgv takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libtgv takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# plain-Python descriptions of the ABI structs
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Bins:
    num_bins: int = 7
    rule: int = 0
    centers: tuple = None      # defaults by rule
    delta: float = None        # world units; default 3 h
    eta_over_delta: float = 3.0

    def to_c(self, h: float) -> BinsT:
        b = BinsT()
        b.num_bins = self.num_bins
        b.rule = self.rule
        if self.centers is None:
            if self.rule == 0:
                c = np.linspace(-1.0, 1.0, self.num_bins) if self.num_bins > 1 else np.zeros(1)
            else:
                c = -1.0 + (2.0 * np.arange(self.num_bins) + 1.0) / self.num_bins
        else:
            c = np.asarray(self.centers, dtype=np.float64)
        cc = np.full(8, np.inf, dtype=np.float32)
        m = max(0, min(self.num_bins, 8))  # an out-of-range count is passed on for the library to reject
        cc[:m] = c[:m].astype(np.float32)
        for k in range(8):
            b.centers[k] = float(cc[k])
        b.delta = float(np.float32(3.0) * np.float32(h)) if self.delta is None else float(self.delta)
        b.eta_over_delta = float(self.eta_over_delta)
        return b

    def centers32(self) -> np.ndarray:
        b = self.to_c(1.0)
        return np.array([b.centers[k] for k in range(8)], dtype=np.float32)


@dataclasses.dataclass
class Params:
    alpha0: float = 2.0
    alpha1: float = 1.0
    lam: float = 1.0
    tau: float = float(1.0 / np.sqrt(12.0))
    sigma: float = float(1.0 / np.sqrt(12.0))
    iters: int = 300
    storage: int = STORE_F32
    schedule: int = SCHED_AUTO
    tile_y: int = 0
    tile_z: int = 0
    flags: int = 0

    def to_c(self) -> ParamsT:
        p = ParamsT()
        p.alpha0, p.alpha1, p.lam = self.alpha0, self.alpha1, self.lam
        p.tau, p.sigma = self.tau, self.sigma
        p.iters, p.storage, p.schedule = int(self.iters), int(self.storage), int(self.schedule)
        p.tile_y, p.tile_z = int(self.tile_y), int(self.tile_z)
        p.flags = int(self.flags)
        return p


def grid_c(origin, h, n, halo=0) -> GridT:
    g = GridT()
    for i in range(3):
        g.origin[i] = float(origin[i])
    g.h = float(h)
    g.nx, g.ny, g.nz = (int(v) for v in n)
    g.halo = int(halo)
    return g


def grid_from(obj) -> GridT:
    """Accepts a GridT or any object with origin, h, n, halo attributes."""
    if isinstance(obj, GridT):
        return obj
    return grid_c(obj.origin, obj.h, obj.n, getattr(obj, "halo", 0))


def cameras_c(R, t, intr, wh, vote, model=None):
    n = int(np.asarray(R).shape[0])
    model = np.zeros(n, dtype=np.int32) if model is None else np.asarray(model, dtype=np.int32).reshape(n)
    arr = (Camera * max(n, 1))()
    R = np.asarray(R, dtype=np.float32).reshape(n, 9)
    t = np.asarray(t, dtype=np.float32).reshape(n, 3)
    intr = np.asarray(intr, dtype=np.float32).reshape(n, 4)
    wh = np.asarray(wh, dtype=np.int32).reshape(n, 2)
    vote = np.asarray(vote, dtype=np.int32).reshape(n)
    for k in range(n):
        c = arr[k]
        for i in range(9):
            c.R[i] = float(R[k, i])
        for i in range(3):
            c.t[i] = float(t[k, i])
        c.fx, c.fy, c.cx, c.cy = (float(v) for v in intr[k])
        c.width, c.height = int(wh[k, 0]), int(wh[k, 1])
        c.vote = int(vote[k])
        c.model = int(model[k])
    return arr, n


def cameras_from(obj):
    """Accepts (array, n) or an object with R, t, intr, wh, vote (and
    optionally model) arrays."""
    if isinstance(obj, tuple):
        return obj
    return cameras_c(obj.R, obj.t, obj.intr, obj.wh, obj.vote, getattr(obj, "model", None))


def stats_dict(s: StatsT) -> dict:
    return dict(primal=s.primal, dual=s.dual, gap_rel=s.gap_rel, parts=[s.parts[0], s.parts[1], s.parts[2]],
                nonfinite=int(s.nonfinite), iters_done=int(s.iters_done))


# ---------------------------------------------------------------------------
# context and calls
# ---------------------------------------------------------------------------
class Context:
    """A libtgv context on one device (owns the library-side workspace)."""

    def __init__(self, device: int = None, lib_path: str = None):
        self.lib = load_library() if lib_path is None else load_library(lib_path)
        if not torch.cuda.is_available():
            raise RuntimeError("libtgv needs a ROCm GPU; torch.cuda.is_available() is False")
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = _vp()
        st = self.lib.tgv_create(self.device, ctypes.byref(h))
        if st != TGV_OK:
            raise TgvError(st, f"tgv_create(device={self.device}) failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tgv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != TGV_OK:
            msg = self.lib.tgv_last_error(self.h)
            raise TgvError(st, msg.decode() if msg else "")

    # -- pyramids ----------------------------------------------------------
    def pyramid_floats(self, W: int, H: int) -> int:
        return int(self.lib.tgv_pyramid_floats(W, H))

    def pyramid_levels(self, W: int, H: int) -> int:
        return int(self.lib.tgv_pyramid_levels(W, H))

    def build_pyramids(self, depth: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        n, H, W = depth.shape
        if depth.dtype != torch.float32:
            raise ValueError("depth maps must be float32")
        if out is None:
            out = torch.empty((n, self.pyramid_floats(W, H)), dtype=torch.float32, device=depth.device)
        self._check(self.lib.tgv_build_pyramids(self.h, _ptr(depth), n, W, H, _ptr(out), _stream(stream)))
        return out

    # -- histograms --------------------------------------------------------
    def cull(self, cams, grid) -> np.ndarray:
        arr, n = cameras_from(cams)
        keep = (ctypes.c_int32 * max(n, 1))()
        g = grid_from(grid)
        cnt = self.lib.tgv_cull_cameras(arr, n, ctypes.byref(g), keep)
        if cnt < 0:
            raise TgvError(TGV_E_INVAL, "tgv_cull_cameras: bad arguments")
        return np.array(keep[:cnt], dtype=np.int32)

    def build_histograms(self, pyr: torch.Tensor, W: int, H: int, cams, grid, bins: Bins = None,
                         out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """uint16 histograms as an int16 tensor [n_voxels, 8] (reinterpret as uint16)."""
        g = grid_from(grid)
        b = (bins or Bins()).to_c(g.h)
        arr, n = cameras_from(cams)
        nvox = g.nx * g.ny * g.nz
        if out is None:
            out = torch.empty((nvox, 8), dtype=torch.int16, device=pyr.device)
        self._check(self.lib.tgv_build_histograms(self.h, _ptr(pyr), W, H, arr, n, ctypes.byref(g), ctypes.byref(b),
                                                  _ptr(out), _stream(stream)))
        return out

    def build_pyramids_mixed(self, depths, stream=None):
        """Pyramids of several stacks of depth maps of different sizes (a list
        of float32 tensors [n_i, H_i, W_i]) packed into one buffer: returns
        (pyr, offsets), offsets[c] the float offset of camera c's pyramid, in
        the order of the stacks."""
        sizes = [(int(d.shape[0]), int(d.shape[2]), int(d.shape[1])) for d in depths]
        total = sum(n * self.pyramid_floats(W, H) for n, W, H in sizes)
        dev = depths[0].device
        pyr = torch.empty(total, dtype=torch.float32, device=dev)
        offsets, at = [], 0
        for d, (n, W, H) in zip(depths, sizes):
            per = self.pyramid_floats(W, H)
            self.build_pyramids(d, out=pyr[at:at + n * per].view(n, per), stream=stream)
            offsets.extend(at + k * per for k in range(n))
            at += n * per
        return pyr, np.asarray(offsets, dtype=np.int64)

    def build_histograms_ex(self, pyr: torch.Tensor, offsets, cams, grid, bins: Bins = None, accumulate: bool = False,
                            prior_votes: int = 0, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """Histograms from cameras of different sizes and models (pinhole maps
        and 360-degree scans), camera c's pyramid at pyr[offsets[c]:]; with
        accumulate, added to out's counts (at most prior_votes per voxel)."""
        g = grid_from(grid)
        b = (bins or Bins()).to_c(g.h)
        arr, n = cameras_from(cams)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        if offs.size != n:
            raise ValueError("one pyramid offset per camera")
        nvox = g.nx * g.ny * g.nz
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs the histograms to add to")
            out = torch.empty((nvox, 8), dtype=torch.int16, device=pyr.device)
        optr = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        self._check(self.lib.tgv_build_histograms_ex(self.h, _ptr(pyr), optr, arr, n, ctypes.byref(g), ctypes.byref(b),
                                                     HIST_ACCUMULATE if accumulate else 0, int(prior_votes),
                                                     _ptr(out), _stream(stream)))
        return out

    # -- solver ------------------------------------------------------------
    def state(self, grid, storage: int = STORE_F32) -> "State":
        return State(self, grid, storage)

    def solve(self, grid, hist: torch.Tensor, u_io: torch.Tensor, params: Params = None, bins: Bins = None,
              state: "State" = None, stats: bool = False, stream=None):
        """Run params.iters iterations; fresh from u_io unless a state is given.
        Returns the stats dict when stats=True (synchronises), else None."""
        g = grid_from(grid)
        p = (params or Params()).to_c()
        b = (bins or Bins()).to_c(g.h)
        s = StatsT()
        self._check(self.lib.tgv_solve(self.h, ctypes.byref(g), _ptr(hist), ctypes.byref(b), ctypes.byref(p),
                                       _ptr(u_io), state.h if state is not None else None,
                                       ctypes.byref(s) if stats else None, _stream(stream)))
        return stats_dict(s) if stats else None

    def solve_noalloc(self, grid, hist: torch.Tensor, u_io: torch.Tensor, params: Params = None, bins: Bins = None,
                      stream=None):
        """Fresh solve whose state lives in the library's fixed device
        workspace (no device allocation; blocks whose state fits in
        NOALLOC_MAX_BYTES).  u_io: initial values in, u out."""
        g = grid_from(grid)
        p = (params or Params()).to_c()
        b = (bins or Bins()).to_c(g.h)
        self._check(self.lib.tgv_solve_noalloc(self.h, ctypes.byref(g), _ptr(hist), ctypes.byref(b), ctypes.byref(p),
                                               _ptr(u_io), _stream(stream)))

    def solve_batch(self, states, hists, params: Params = None, bins: Bins = None, tile_z=None, stats: bool = False,
                    stream=None):
        """Advance every state by params.iters iterations in batched launches
        (bit-identical to solving each alone).  hists: device tensors, one per
        state.  tile_z: optional per-block z-chunk list.  Returns per-block
        stats when stats=True (synchronises)."""
        n = len(states)
        if len(hists) != n:
            raise ValueError("one histogram tensor per state")
        p = (params or Params()).to_c()
        b = (bins or Bins()).to_c(states[0].grid.h if n else 1.0)
        sarr = (_vp * max(n, 1))(*[s.h for s in states])
        harr = (_vp * max(n, 1))(*[_ptr(h) for h in hists])
        tz = None
        if tile_z is not None:
            tz = (ctypes.c_int32 * max(n, 1))(*[int(v) for v in tile_z])
        st = (StatsT * max(n, 1))()
        self._check(self.lib.tgv_solve_batch(self.h, n, sarr, harr, ctypes.byref(b), ctypes.byref(p), tz,
                                             st if stats else None, _stream(stream)))
        return [stats_dict(st[i]) for i in range(n)] if stats else None

    def prolongate(self, coarse, u_coarse: torch.Tensor, fine, out: torch.Tensor = None, stream=None):
        gc, gf = grid_from(coarse), grid_from(fine)
        if out is None:
            out = torch.empty(gf.nx * gf.ny * gf.nz, dtype=torch.float32, device=u_coarse.device)
        self._check(self.lib.tgv_prolongate(self.h, ctypes.byref(gc), _ptr(u_coarse), ctypes.byref(gf), _ptr(out),
                                            _stream(stream)))
        return out

    def solve_coarse_to_fine(self, pyr: torch.Tensor, W: int, H: int, cams, grid, levels: int,
                             params: Params = None, bins: Bins = None, stream=None) -> torch.Tensor:
        """Coarse-to-fine solve of one block; returns the finest u."""
        g = grid_from(grid)
        b = (bins or Bins()).to_c(g.h)
        p = (params or Params(iters=200)).to_c()
        arr, n = cameras_from(cams)
        out = torch.empty(g.nx * g.ny * g.nz, dtype=torch.float32, device=pyr.device)
        self._check(self.lib.tgv_solve_coarse_to_fine(self.h, _ptr(pyr), W, H, arr, n, ctypes.byref(g),
                                                      ctypes.byref(b), ctypes.byref(p), int(levels), _ptr(out),
                                                      _stream(stream)))
        return out

    def extract_crossings(self, grid, u: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """Zero-level points of u as a float32 tensor [count, 4] (X, Y, Z, axis).
        With `out` ([capacity, 4] float32) one call fills it and returns its
        first count rows (a ValueError if the points do not fit); without, a
        counting call sizes the output first."""
        g = grid_from(grid)
        cnt = ctypes.c_int64()
        if out is not None:
            if out.dtype != torch.float32 or out.dim() != 2 or out.shape[1] != 4:
                raise ValueError("out must be a float32 tensor [capacity, 4]")
            self._check(self.lib.tgv_extract_crossings(self.h, ctypes.byref(g), _ptr(u), _ptr(out), out.shape[0],
                                                       ctypes.byref(cnt), _stream(stream)))
            if cnt.value > out.shape[0]:
                raise ValueError(f"{cnt.value} points do not fit in {out.shape[0]} rows")
            return out[:cnt.value]
        self._check(self.lib.tgv_extract_crossings(self.h, ctypes.byref(g), _ptr(u), None, 0, ctypes.byref(cnt),
                                                   _stream(stream)))
        out = torch.empty((max(cnt.value, 1), 4), dtype=torch.float32, device=u.device)
        self._check(self.lib.tgv_extract_crossings(self.h, ctypes.byref(g), _ptr(u), _ptr(out), cnt.value,
                                                   ctypes.byref(cnt), _stream(stream)))
        return out[:cnt.value]

    def stream_copy(self, src: torch.Tensor, dst: torch.Tensor, variant: int = 0, stream=None):
        """Plain streaming copy of src into dst (same byte size, a multiple of
        16) by the library's copy kernel of the given shape (see
        tgv_stream_copy)."""
        nbytes = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nbytes:
            raise ValueError("src and dst differ in size")
        self._check(self.lib.tgv_stream_copy(self.h, _ptr(src), _ptr(dst), nbytes, int(variant), _stream(stream)))

    def energy(self, state: "State", hist: torch.Tensor, params: Params = None, bins: Bins = None,
               stream=None) -> dict:
        p = (params or Params()).to_c()
        b = (bins or Bins()).to_c(state.grid.h)
        s = StatsT()
        self._check(self.lib.tgv_energy(self.h, state.h, _ptr(hist), ctypes.byref(b), ctypes.byref(p),
                                        ctypes.byref(s), _stream(stream)))
        return stats_dict(s)


def state_bytes(grid, storage: int = STORE_F32) -> int:
    """Device bytes of a solver state (-1 for an invalid grid)."""
    g = grid_from(grid)
    return int(load_library().tgv_state_bytes(ctypes.byref(g), storage))


class State:
    """A resumable solver state: device memory owned by libtgv, or a torch
    tensor given as `memory` (kept alive by this object)."""

    def __init__(self, ctx: Context, grid, storage: int = STORE_F32, memory: torch.Tensor = None):
        self.ctx = ctx
        self.grid = grid_from(grid)
        self.storage = storage
        self.memory = memory
        h = _vp()
        if memory is None:
            ctx._check(ctx.lib.tgv_state_create(ctx.h, ctypes.byref(self.grid), storage, ctypes.byref(h)))
        else:
            ctx._check(ctx.lib.tgv_state_wrap(ctx.h, ctypes.byref(self.grid), storage, _ptr(memory),
                                              memory.numel() * memory.element_size(), ctypes.byref(h)))
        self.h = h
        self.n = self.grid.nx * self.grid.ny * self.grid.nz

    def bytes(self) -> int:
        return int(self.ctx.lib.tgv_state_bytes(ctypes.byref(self.grid), self.storage))

    def reset(self, u0: torch.Tensor, stream=None):
        self.ctx._check(self.ctx.lib.tgv_state_reset(self.ctx.h, self.h, _ptr(u0), _stream(stream)))

    def export(self, stream=None, fields=("u", "v", "u_prev", "v_prev", "p", "q")) -> dict:
        dev = torch.device("cuda", self.ctx.device)
        n = self.n
        size = dict(u=n, v=3 * n, u_prev=n, v_prev=3 * n, p=3 * n, q=6 * n)
        out = {f: torch.empty(size[f], device=dev) for f in fields}
        self.ctx._check(self.ctx.lib.tgv_state_export(self.ctx.h, self.h, _ptr(out.get("u")), _ptr(out.get("v")),
                                                      _ptr(out.get("u_prev")), _ptr(out.get("v_prev")),
                                                      _ptr(out.get("p")), _ptr(out.get("q")), _stream(stream)))
        return out

    def import_(self, f: dict, iters_done: int = 0, stream=None):
        self.ctx._check(self.ctx.lib.tgv_state_import(self.ctx.h, self.h, _ptr(f["u"]), _ptr(f["v"]),
                                                      _ptr(f["u_prev"]), _ptr(f["v_prev"]), _ptr(f["p"]),
                                                      _ptr(f["q"]), int(iters_done), _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tgv_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
