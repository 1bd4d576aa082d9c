"""The batched-solve autotuner's search without a GPU: class grouping,
candidate shapes, the choice of (schedule, tile_y) by the time summed over
classes, per-class tile_z, and the cache.  A cost model stands in for the
device timing."""
import json

import pytest

from paper_2107_14790_amd import autotune


class G:
    def __init__(self, n):
        self.n = n


def test_edge_classes():
    assert autotune.edge_class((36, 36, 36)) == 0
    assert autotune.edge_class((48, 10, 10)) == 0
    assert autotune.edge_class((49, 10, 10)) == 1
    assert autotune.edge_class((10, 10, 128)) == 2
    assert autotune.edge_class((196, 196, 196)) == 4


def test_candidates_cover_both_schedules_and_skip_deep_chunks():
    c = autotune.candidates([(40, 40, 20)])
    assert ("fused", 8, 8) in c and ("fused2", 7, 32) in c
    assert all(tz <= 40 or tz == 8 for _, _, tz in c)
    assert {s for s, _, _ in c} == {"fused", "fused2"}
    assert {ty for s, ty, _ in c if s == "fused2"} == {4, 6, 7}


def model(best_small, best_big):
    """ms: class of edge <= 48 is fastest at best_small, others at best_big;
    every shape's time grows with its voxels."""
    calls = []

    def measure(shapes, storage, sched, ty, tz):
        calls.append((tuple(shapes), sched, ty, tz))
        vox = sum(a * b * c for a, b, c in shapes)
        small = max(max(s) for s in shapes) <= 48
        target = best_small if small else best_big
        miss = (sched != target[0]) * 3 + abs(ty - target[1]) * 0.5 + abs(tz - target[2]) / 16
        return vox * 1e-6 * (1 + miss)
    return measure, calls


def test_pick_follows_the_voxel_weighted_sum():
    # many small blocks prefer fused 4x16; a few large ones prefer fused2 7x32.
    # The large blocks hold most voxels, so the batch runs fused2 at tile_y 7,
    # and the small class takes its best tile_z at that pair.
    grids = [G((36, 36, 36))] * 40 + [G((120, 120, 120))] * 6
    measure, calls = model(("fused", 4, 16), ("fused2", 7, 32))
    t = autotune.Autotuner(measure=measure, device_name="model")
    r = t.tune(grids)
    assert r["schedule"] == "fused2" and r["tile_y"] == 7
    assert r["tile_z"][0] == 16 and r["tile_z"][-1] == 32
    assert len(r["tile_z"]) == len(grids)
    # with the voxels the other way round the small blocks' choice wins
    grids2 = [G((44, 44, 44))] * 400 + [G((60, 60, 60))] * 2
    measure2, _ = model(("fused", 4, 16), ("fused2", 7, 32))
    r2 = autotune.Autotuner(measure=measure2, device_name="model").tune(grids2)
    assert r2["schedule"] == "fused" and r2["tile_y"] == 4 and r2["tile_z"][0] == 16


def test_samples_at_most_16_blocks_per_class_and_caches(tmp_path):
    grids = [G((30 + i % 9, 40, 41)) for i in range(50)]
    measure, calls = model(("fused2", 6, 8), ("fused2", 6, 8))
    path = str(tmp_path / "tune.json")
    t = autotune.Autotuner(measure=measure, device_name="model", cache_path=path)
    r = t.tune(grids)
    assert r["schedule"] == "fused2" and r["tile_y"] == 6 and set(r["tile_z"]) == {8}
    assert all(len(c[0]) == 16 for c in calls)
    n_calls = len(calls)
    assert n_calls == len(autotune.candidates([c for c in calls[0][0]]))
    saved = json.load(open(path))
    assert any(k.startswith("model|s0|c0") for k in saved)
    # a second tuner reads the cache and measures nothing
    measure3, calls3 = model(("fused", 4, 8), ("fused", 4, 8))
    r3 = autotune.Autotuner(measure=measure3, device_name="model", cache_path=path).tune(grids)
    assert calls3 == [] and r3["schedule"] == "fused2"


def test_pick_ignores_pairs_missing_on_a_class():
    per_class = {0: {"all": {"fused,4,8": 1.0, "fused2,7,8": 0.5}},
                 1: {"all": {"fused,4,8": 2.0}}}
    r = autotune.pick(per_class, {0: 1.0, 1: 1.0})
    assert r["schedule"] == "fused" and r["tile_y"] == 4


def test_class_wise_choice_is_checked_on_the_batch():
    """Timed alone, small blocks want short chunks (they fill the chip); in
    the mixed batch short chunks only add halo planes.  The check on a
    sample of the batch takes the faster alternative, and the library
    default when it beats every tuned variant."""
    grids = [G((36, 36, 36))] * 40 + [G((120, 120, 120))] * 6
    measure, _ = model(("fused2", 7, 8), ("fused2", 7, 32))
    mixes = []

    def mix_deep(shapes, storage, sched, ty, tz):
        # four halo planes per chunk; a chunk deeper than its block is the block
        mixes.append((len(shapes), sched, ty, None if tz is None else tuple(tz)))
        vox = sum(a * b * c for a, b, c in shapes)
        if tz is None:
            return vox * 1e-6 * 1.15
        halo = sum(a * b * c * 4.0 / min(t, c) for (a, b, c), t in zip(shapes, tz))
        return (vox + halo) * 1e-6

    r = autotune.Autotuner(measure=measure, measure_mix=mix_deep, device_name="model").tune(grids)
    assert r["schedule"] == "fused2" and r["tile_y"] == 7
    assert r["checked_on_batch"]["chosen"] == "uniform chunks of 128"
    assert r["tile_z"] == [128] * len(grids)
    assert all(n == len(grids) for n, _, _, _ in mixes) and len(mixes) == 7
    ms = r["checked_on_batch"]["ms"]
    # deeper chunks of the class-wise choice are faster in this model, the
    # tuned shapes beat the default, and the fastest alternative is taken
    assert ms["class-wise"] > ms["class-wise, chunks doubled"] > ms["class-wise, chunks quadrupled"]
    assert min(ms, key=ms.get) == "uniform chunks of 128"

    def mix_doubled(shapes, storage, sched, ty, tz):
        # the doubled class-wise chunks are the fastest shape of this batch
        vox = sum(a * b * c for a, b, c in shapes)
        if tz is None:
            return vox * 1e-6 * 1.15
        want = [min(2 * (8 if c <= 48 else 32), 128) for (a, b, c) in shapes]
        return vox * 1e-6 * (1.0 if list(tz) == want else 1.1)

    r1 = autotune.Autotuner(measure=measure, measure_mix=mix_doubled, device_name="model").tune(grids)
    assert r1["checked_on_batch"]["chosen"] == "class-wise, chunks doubled"
    assert r1["tile_z"][0] == 16 and r1["tile_z"][-1] == 64

    def mix_default(shapes, storage, sched, ty, tz):
        vox = sum(a * b * c for a, b, c in shapes)
        return vox * 1e-6 * (0.9 if tz is None else 1.0)

    r2 = autotune.Autotuner(measure=measure, measure_mix=mix_default, device_name="model").tune(grids)
    assert r2["checked_on_batch"]["chosen"] == "library default"
    assert r2["schedule"] == "fused2" and r2["tile_y"] == 7 and r2["tile_z"] is None
