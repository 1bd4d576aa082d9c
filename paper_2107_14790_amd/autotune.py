"""Schedule and tile-shape autotuner for batched TGV solves.

A batched solve runs either one fused iteration per persistent launch
(schedule FUSED, tiles of 64 x tile_y columns with tile_y in {4, 8, 12}) or
two (schedule FUSED2, temporal blocking, tile_y in {4, 6, 7}); each block's
tiles walk chunks of tile_z planes.  tile_y is a kernel template parameter,
so it is one per batch; tile_z is per block.  The best choice depends on
the block sizes (how many tiles fill the chip, how much of each chunk is
halo) and on the storage precision.

The autotuner groups blocks into padded-edge classes, times every candidate
(schedule, tile_y, tile_z) on a representative batch of each class through
the batched C-ABI call (synthetic histograms, a few iterations), then picks
the (schedule, tile_y) whose time summed over the classes (each scaled from
its sample to the class's voxels) is least, and for each class the tile_z
that is fastest at that pair.  A class timed alone is not the batch: in the
mix the work queue has tiles to spare, and short chunks that fill the chip
for one class only add halo planes there.  So the class-wise choice is
checked on a sample of the batch itself against a few alternatives (the
same pair with chunks two or four times deeper, or uniform chunks of 32, 64
or 128 planes, and the library's default) and the fastest of them is taken.  Results are cached per device, storage and
class.  The measurements are function arguments, so the search itself runs
without a GPU (tests give it a model).
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, List, Sequence

import numpy as np

SCHED_NAMES = ("fused", "fused2")
TILE_Y = {"fused": (4, 8, 12), "fused2": (4, 6, 7)}
TILE_Z = (8, 16, 32, 64, 128)
CLASS_EDGES = (48, 80, 128, 192, 1 << 30)  # padded edge upper bounds of the classes
TUNE_ITERS = 9  # one dual step, four two-iteration launches (or eight one-iteration ones), one primal step
MIX_BLOCKS = 96  # blocks of the batch sample the class-wise choice is checked on


def edge_class(n: Sequence[int]) -> int:
    e = max(int(v) for v in n)
    for k, b in enumerate(CLASS_EDGES):
        if e <= b:
            return k
    return len(CLASS_EDGES) - 1


def candidates(shapes: Sequence[Sequence[int]]):
    """(schedule, tile_y, tile_z) triples worth timing on blocks of these shapes:
    chunks deeper than twice the deepest block are the same as the block."""
    zmax = max(int(v[2]) for v in shapes)
    out = []
    for sched in SCHED_NAMES:
        for ty in TILE_Y[sched]:
            for tz in TILE_Z:
                if tz <= 2 * zmax or tz == TILE_Z[0]:
                    out.append((sched, ty, tz))
    return out


def pick(per_class: Dict[int, dict], weight: Dict[int, float], schedules=SCHED_NAMES) -> dict:
    """Choose (schedule, tile_y) minimising the weighted sum over classes of
    each class's best time at that pair, then each class's tile_z there.
    per_class[c]["all"] maps "sched,ty,tz" to ms on the class's sample;
    weight[c] scales the sample to the class's share of the batch; only the
    given schedules are considered."""
    pairs = {}
    for cls, r in per_class.items():
        for key, ms in r["all"].items():
            sched, ty, _ = key.split(",")
            if sched not in schedules:
                continue
            pairs.setdefault((sched, int(ty)), {}).setdefault(cls, []).append(ms)
    total = {}
    for pair, by_cls in pairs.items():
        if set(by_cls) != set(per_class):
            continue  # a pair not timed on every class
        total[pair] = sum(weight[c] * min(v) for c, v in by_cls.items())
    sched, ty = min(total, key=total.get)
    tz_of = {}
    for cls, r in per_class.items():
        cands = {k: v for k, v in r["all"].items() if k.startswith(f"{sched},{ty},")}
        tz_of[cls] = int(min(cands, key=cands.get).split(",")[2])
    return {"schedule": sched, "tile_y": ty, "tile_z_of_class": tz_of, "predicted_ms": total[(sched, ty)]}


class Autotuner:
    def __init__(self, ctx=None, cache_path: str = None, iters: int = TUNE_ITERS, reps: int = 3,
                 measure: Callable = None, device_name: str = None, measure_mix: Callable = None):
        """ctx: a libtgv Context (None when a `measure` model is given).
        measure(shapes, storage, schedule, tile_y, tile_z) -> ms replaces the
        GPU timing of a class sample, measure_mix(shapes, storage, schedule,
        tile_y, tile_z_list or None) -> ms that of a batch sample (for tests;
        with a `measure` model and no `measure_mix` the check on the batch
        is skipped)."""
        self.ctx = ctx
        self.iters = iters
        self.reps = reps
        self.cache_path = cache_path
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)
        self.measure = measure or self._gpu_measure
        self.measure_mix = measure_mix or (None if measure else self._gpu_measure_mix)
        if device_name is None:
            import torch
            device_name = torch.cuda.get_device_name(ctx.device)
        self.device_name = device_name
        self._batch = None

    def _key(self, storage: int, cls: int) -> str:
        return f"{self.device_name}|s{storage}|c{cls}|v2"

    # -- GPU measurement ---------------------------------------------------
    def _gpu_measure(self, shapes, storage, sched, ty, tz) -> float:
        import torch
        import paper_2107_14790_amd as tgv
        key = (tuple(tuple(s) for s in shapes), storage)
        if self._batch is None or self._batch[0] != key:
            self._release()
            states, hists = [], []
            for n in shapes:
                g = tgv.grid_c((0, 0, 0), 1.0, n, min(2, (min(n) - 1) // 2))
                st = tgv.State(self.ctx, g, storage)
                nv = int(np.prod(n))
                st.reset(torch.zeros(nv, device="cuda"))
                h = torch.zeros((nv, 8), dtype=torch.int16, device="cuda")
                h[:, 6] = 1
                states.append(st)
                hists.append(h)
            self._batch = (key, states, hists)
        _, states, hists = self._batch
        p = tgv.Params(iters=self.iters, storage=storage, tile_y=ty, tile_z=tz,
                       schedule=tgv.SCHED_FUSED2 if sched == "fused2" else tgv.SCHED_FUSED)
        s = torch.cuda.current_stream()
        self.ctx.solve_batch(states, hists, p, tile_z=[tz] * len(states))  # warm
        best = float("inf")
        for _ in range(self.reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            self.ctx.solve_batch(states, hists, p, tile_z=[tz] * len(states))
            e1.record(s)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def _gpu_measure_mix(self, shapes, storage, sched, ty, tz_list) -> float:
        """Time one batched solve of these shapes with per-block chunks
        (None: the library's default)."""
        import torch
        import paper_2107_14790_amd as tgv
        key = (tuple(tuple(s) for s in shapes), storage)
        if self._batch is None or self._batch[0] != key:
            self.measure(shapes, storage, sched, ty, 32)  # builds the sample's states
        _, states, hists = self._batch
        p = tgv.Params(iters=self.iters, storage=storage, tile_y=ty,
                       schedule=tgv.SCHED_FUSED2 if sched == "fused2" else tgv.SCHED_FUSED)
        s = torch.cuda.current_stream()
        self.ctx.solve_batch(states, hists, p, tile_z=tz_list)  # warm
        best = float("inf")
        for _ in range(self.reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            self.ctx.solve_batch(states, hists, p, tile_z=tz_list)
            e1.record(s)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def _release(self):
        if self._batch is not None:
            for st in self._batch[1]:
                st.close()
            self._batch = None

    # -- search ------------------------------------------------------------
    def tune_class(self, shapes: List[Sequence[int]], storage: int = 0, max_blocks: int = 16) -> dict:
        """Time every candidate on up to max_blocks representative shapes of one class."""
        rng = np.random.default_rng(0)
        sample = [tuple(int(v) for v in shapes[i])
                  for i in rng.choice(len(shapes), size=min(len(shapes), max_blocks), replace=False)]
        res = {}
        for sched, ty, tz in candidates(sample):
            res[f"{sched},{ty},{tz}"] = float(self.measure(sample, storage, sched, ty, tz))
        self._release()
        best = min(res, key=res.get)
        return {"best": best, "ms": res[best], "all": res,
                "sample_voxels": int(sum(int(np.prod(s)) for s in sample))}

    def tune(self, grids, storage: int = 0) -> dict:
        """Schedule, batch-wide tile_y and per-block tile_z for a list of block
        grids (objects with an `n` attribute)."""
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
        weight = {cls: sum(int(np.prod(s)) for s in shapes) / per_class[cls]["sample_voxels"]
                  for cls, shapes in classes.items()}
        choice = pick(per_class, weight)
        tile_z = [choice["tile_z_of_class"][edge_class(g.n)] for g in grids]
        best_sched, best_ty = choice["schedule"], choice["tile_y"]
        checked = None
        if self.measure_mix is not None:
            # the class-wise choice against alternatives, on a sample of the batch
            rng = np.random.default_rng(1)
            idx = sorted(rng.choice(len(grids), size=min(len(grids), MIX_BLOCKS), replace=False).tolist())
            shapes = [tuple(int(v) for v in grids[i].n) for i in idx]
            tz_class = choice["tile_z_of_class"]
            # each alternative: schedule, tile_y and a block's tile_z (None: the library's default)
            deep = lambda k: (lambda n: min(k * tz_class[edge_class(n)], TILE_Z[-1]))
            uniform = lambda tz: (lambda n: tz)
            alts = {
                "class-wise": (best_sched, best_ty, deep(1)),
                "class-wise, chunks doubled": (best_sched, best_ty, deep(2)),
                "class-wise, chunks quadrupled": (best_sched, best_ty, deep(4)),
                "uniform chunks of 32": (best_sched, best_ty, uniform(32)),
                "uniform chunks of 64": (best_sched, best_ty, uniform(64)),
                "uniform chunks of 128": (best_sched, best_ty, uniform(128)),
                "library default": ("fused2", 7, None),
            }
            checked = {name: float(self.measure_mix(shapes, storage, a, b, None if f is None else [f(n) for n in shapes]))
                       for name, (a, b, f) in alts.items()}
            self._release()
            win = min(checked, key=checked.get)
            best_sched, best_ty, f = alts[win]
            tile_z = None if f is None else [f(tuple(int(v) for v in g.n)) for g in grids]
            checked = {"sample_blocks": len(shapes), "ms": checked, "chosen": win}
        by_schedule = {}
        for sched in SCHED_NAMES:
            c = pick(per_class, weight, (sched,))
            by_schedule[sched] = {"tile_y": c["tile_y"], "predicted_ms": c["predicted_ms"],
                                  "tile_z": [c["tile_z_of_class"][edge_class(g.n)] for g in grids]}
        return {"schedule": best_sched, "tile_y": best_ty, "tile_z": tile_z, "checked_on_batch": checked,
                "predicted_ms": choice["predicted_ms"], "by_schedule": by_schedule,
                "classes": {str(k): {"best": v["best"], "ms": v["ms"], "tile_z": choice["tile_z_of_class"][k]}
                            for k, v in per_class.items()}}

    @staticmethod
    def params(tuned: dict, iters: int, storage: int = 0, flags: int = 0):
        """Batched-solve parameters for a tune() result."""
        import paper_2107_14790_amd as tgv
        return tgv.Params(iters=iters, storage=storage, tile_y=tuned["tile_y"], flags=flags,
                          schedule=tgv.SCHED_FUSED2 if tuned["schedule"] == "fused2" else tgv.SCHED_FUSED)
