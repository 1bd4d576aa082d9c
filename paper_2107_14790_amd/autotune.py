"""Tile-shape autotuner for the fused TGV kernel.

The fused kernel walks 64 x tile_y column tiles through chunks of tile_z
planes.  The best shape depends on the block size (how many tiles fill the
chip, how much of each chunk is halo) and on the storage precision.  The
autotuner groups blocks into edge-size classes, times candidate shapes on
the device through the batched C-ABI call (one representative batch per
class, synthetic histograms, a few iterations) and keeps the fastest:
tile_y for the whole batch (it is a kernel template parameter) and tile_z
per class.  Results are cached in a JSON file keyed by device, storage and
class.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Sequence

import numpy as np
import torch

TILE_Y = (4, 8, 12)
TILE_Z = (8, 16, 32, 64, 128)
CLASS_EDGES = (48, 80, 128, 192, 1 << 30)  # padded edge upper bounds of the classes


def edge_class(n: Sequence[int]) -> int:
    e = max(int(v) for v in n)
    for k, b in enumerate(CLASS_EDGES):
        if e <= b:
            return k
    return len(CLASS_EDGES) - 1


class Autotuner:
    def __init__(self, ctx, cache_path: str = None, iters: int = 8, reps: int = 3):
        self.ctx = ctx
        self.iters = iters
        self.reps = reps
        self.cache_path = cache_path
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)
        self.device_name = torch.cuda.get_device_name(ctx.device)

    def _key(self, storage: int, cls: int) -> str:
        return f"{self.device_name}|s{storage}|c{cls}"

    def _time(self, states, hists, params) -> float:
        s = torch.cuda.current_stream()
        best = float("inf")
        for _ in range(self.reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            self.ctx.solve_batch(states, hists, params, tile_z=[params.tile_z] * len(states))
            e1.record(s)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def tune_class(self, shapes: List[Sequence[int]], storage: int = 0, halo: int = 2, max_blocks: int = 16) -> dict:
        """Time every candidate on up to max_blocks representative shapes of one class."""
        import paper_2107_14790_amd as tgv
        rng = np.random.default_rng(0)
        pick = [shapes[i] for i in rng.choice(len(shapes), size=min(len(shapes), max_blocks), replace=False)]
        states, hists = [], []
        for n in pick:
            g = tgv.grid_c((0, 0, 0), 1.0, n, min(halo, (min(n) - 1) // 2))
            st = tgv.State(self.ctx, g, storage)
            nv = int(np.prod(n))
            st.reset(torch.zeros(nv, device="cuda"))
            h = torch.zeros((nv, 8), dtype=torch.int16, device="cuda")
            h[:, 6] = 1
            states.append(st)
            hists.append(h)
        res = {}
        for ty in TILE_Y:
            for tz in TILE_Z:
                if tz > 2 * max(int(v[2]) for v in pick):
                    continue
                p = tgv.Params(iters=self.iters, storage=storage, tile_y=ty, tile_z=tz)
                self._time(states, hists, p)  # warm
                res[f"{ty},{tz}"] = self._time(states, hists, p)
        for st in states:
            st.close()
        best = min(res, key=res.get)
        ty, tz = (int(v) for v in best.split(","))
        return {"tile_y": ty, "tile_z": tz, "ms": res[best], "all": res}

    def tune(self, grids, storage: int = 0) -> dict:
        """Per-class tile_z and one batch-wide tile_y for a list of block grids."""
        classes: Dict[int, list] = {}
        for g in grids:
            n = tuple(int(v) for v in g.n)
            classes.setdefault(edge_class(n), []).append(n)
        per_class = {}
        for cls, shapes in sorted(classes.items()):
            key = self._key(storage, cls)
            if key not in self.cache:
                t0 = time.perf_counter()
                self.cache[key] = self.tune_class(shapes, storage)
                self.cache[key]["tune_s"] = time.perf_counter() - t0
            per_class[cls] = self.cache[key]
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        # tile_y: the class holding most voxels decides; tile_z: each class its best at that tile_y
        weight = {cls: sum(int(np.prod(s)) for s in shapes) for cls, shapes in classes.items()}
        main = max(weight, key=weight.get)
        ty = per_class[main]["tile_y"]
        tz_of = {}
        for cls, r in per_class.items():
            cands = {k: v for k, v in r["all"].items() if int(k.split(",")[0]) == ty}
            tz_of[cls] = int(min(cands, key=cands.get).split(",")[1])
        tile_z = [tz_of[edge_class(g.n)] for g in grids]
        return {"tile_y": ty, "tile_z": tile_z, "classes": {str(k): v for k, v in per_class.items()}}
