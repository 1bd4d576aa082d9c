"""Benchmark of the depth-map fusion hot path on one MI355X.

One step = the whole path on one voxel block: depth-map pyramids, camera
cull, voxel histograms, state init, `iters` TGV primal-dual iterations and
the float64 energy/gap reduction.  Workload (default): a 256^3 block over
the unit cube fusing 64 nadir 1024x1024 depth maps of a seeded fBm terrain
(Hurst 0.8, amplitude 0.2), depth noise 0.3 voxel, 1 % outliers, 7 bins,
alpha1 = 1, alpha0 = 2, lambda = 1, tau = sigma = 1/sqrt(12), 1000 iterations.

The schedule is the library's default (`--schedule auto`): on a block this
size the iterations run two per pass over HBM (FUSED2, the fastest here);
on the 32^3 sphere block, one tiled pass per iteration.  `--schedule fused`
or `fused2` forces one.

Prints one JSON line (rank 0) with throughput in voxel-updates/s, the
roofline of the dominant kernel (the two-iteration pass: one pass's
algorithmic bytes per launch) measured with HIP events on the stream the
library launches on, the same for the one-iteration kernel on the same
block (`one_pass_kernel`), and the CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "TGV voxel-updates/s + % HBM roofline; p50/p99 block-solve latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def fused_bytes_per_voxel(storage: int) -> int:
    """HBM bytes one pass of the rotated fused kernel moves per voxel: read u,
    v(3), p(3), q(6) and the 16-byte histogram; write u, v, p, q (the
    over-relaxed u and v stay in registers)."""
    fb = 4 if storage == 0 else 2
    state = 4 + 12 * fb  # u + v, p, q (3 + 3 + 6 components)
    return state + 16 + state


def bytes_per_update(storage: int) -> int:
    """Algorithmic HBM bytes of one voxel-update of the plain fused step:
    read u, ubar, v(3), vbar(3), p(3), q(6) and the histogram (16 B), write
    all but the histogram: 152 B with float32 storage, 92 B with v, vbar, p,
    q in 16 bits.  The roofline's `achieved` is this figure times the
    updates a launch performs, over the launch's time."""
    fb = 4 if storage == 0 else 2
    fields = 4 + 4 + 15 * fb  # u, ubar + v, vbar, p, q (15 components)
    return fields + 16 + fields


# per kernel: the committed counter summary and the sources it was taken on
TRAFFIC = {
    "fused": ("tgv_fused_tiled_terrain256_traffic.json",
              ("paper_2107_14790_amd/csrc/solver_tiled.hip", "paper_2107_14790_amd/csrc/device_math.h",
               "paper_2107_14790_amd/csrc/fields.h", "paper_2107_14790_amd/csrc/internal.h")),
    "fused2": ("tgv_fused2_tiled_terrain256_traffic.json",
               ("paper_2107_14790_amd/csrc/solver_tiled2.hip", "paper_2107_14790_amd/csrc/device_math.h",
                "paper_2107_14790_amd/csrc/fields.h", "paper_2107_14790_amd/csrc/internal.h")),
}


def kernel_sources_hash(kernel: str = "fused") -> str:
    import hashlib
    hsh = hashlib.sha256()
    for f in TRAFFIC[kernel][1]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def measured_traffic(storage: int, tile: str, kernel: str = "fused"):
    """HBM bytes per launch of a solver kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size),
    or None if the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", TRAFFIC[kernel][0])
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if (t.get("kernel_sources_sha256") != kernel_sources_hash(kernel) or t.get("storage") != storage
            or t.get("tile") != tile):
        return None
    return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]


def hist_valu_instructions():
    """VALU wave-instructions of one histogram launch on the terrain256
    workload, from the committed counter summary, or None if the kernel's
    source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_hist_terrain256_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    with open(os.path.join(ROOT, "paper_2107_14790_amd/csrc/pyramid_hist.hip"), "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()
    return t["SQ_INSTS_VALU"] if t.get("kernel_source_sha256") == h else None


def cpu_baseline(scene, bins_centers, iters_sample: int = 150, crop: int = 64, nvox_hist: int = 20000):
    """The oracle timed on a bounded sample of the workload (single thread)."""
    import oracle
    t0 = time.perf_counter()
    pyr = oracle.pyramids(scene.depth)
    t_pyr = time.perf_counter() - t0
    g = scene.grid
    nx, ny, nz = g.n
    rng = np.random.default_rng(0)
    vox = rng.choice(g.nvox, size=nvox_hist, replace=False)
    t0 = time.perf_counter()
    oracle.histograms(scene, pyr, vox=vox)
    t_hist = time.perf_counter() - t0
    pairs_s = nvox_hist * len(scene.cams) / t_hist
    # a crop block around mid-height, where the surface is
    import scenes
    o = g.origin.astype(np.float64)
    z0 = max(0, nz // 2 - crop // 2)
    cg = scenes.Grid(np.array([o[0], o[1], o[2] + z0 * g.h], dtype=np.float32), g.h, (crop, crop, crop), 0)
    csc = scenes.Scene(scene.depth, scene.cams, cg)
    hcrop, _ = oracle.histograms(csc, pyr)
    t0 = time.perf_counter()
    oracle.solve(hcrop, (crop, crop, crop), bins_centers, iters_sample)
    t_solve = time.perf_counter() - t0
    ups = crop ** 3 * iters_sample / t_solve
    # the same sample with the oracle's per-voxel loops on the host's cores
    # (bit-identical to the serial run; at most 16 threads, the host share
    # of one GPU)
    k = max(1, min(16, os.cpu_count() or 1))
    with oracle.threads(k):
        t0 = time.perf_counter()
        oracle.histograms(scene, pyr, vox=vox)
        t_hist_k = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.solve(hcrop, (crop, crop, crop), bins_centers, iters_sample)
        t_solve_k = time.perf_counter() - t0
    return dict(value=ups, unit="voxel-updates/s", cores=1, kind="oracle",
                sample=f"oracle float64 solve of a {crop}^3 crop of the block (mid-height), {iters_sample} "
                       f"iterations, {t_solve:.1f} s; oracle histograms {pairs_s:.3g} pairs/s on "
                       f"{nvox_hist} random voxels x {len(scene.cams)} cameras; pyramids {t_pyr:.1f} s",
                hist_pairs_per_s=pairs_s,
                all_cores={"value": crop ** 3 * iters_sample / t_solve_k, "unit": "voxel-updates/s", "cores": k,
                           "hist_pairs_per_s": nvox_hist * len(scene.cams) / t_hist_k,
                           "sample": "the same sample, the oracle's per-voxel loops on k threads"})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="terrain256",
                    choices=["terrain256", "sphere32", "city_batch", "city_serve", "city_precision", "next"])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "fused", "fused2"],
                    help="auto (the library's default): two fused iterations per pass for a block whose iteration "
                         "moves more than 48 MiB and for batches, one per pass otherwise")
    ap.add_argument("--blocks", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--arrivals", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true", help="city_precision: skip the whole-block float64 oracle")
    ap.add_argument("--kernel-only", action="store_true", help="skip the per-kernel roofline timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, copy 1 GiB once (a plain copy of known size for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (one process per GPU, blocks are independent); --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload in ("city_batch", "city_serve", "city_precision") and args.schedule == "auto":
        args.schedule = "fused2"  # the library's choice for batches and for the 384^3 block
    if args.workload == "next":
        return bench_next(args)
    if args.workload == "city_batch":
        return bench_city_batch(args)
    if args.workload == "city_serve":
        return bench_city_serve(args)
    if args.workload == "city_precision":
        return bench_city_precision(args)
    if args.iters is None:
        args.iters = 300 if args.workload == "sphere32" else 1000
    return bench_block(args)


def bench_block(args):
    """One block: terrain256 (the default) or sphere32."""
    import torch
    import paper_2107_14790_amd as tgv
    import scenes

    rank = int(os.environ.get("RANK", "0"))
    dev = torch.device("cuda", 0)
    storage = tgv.STORAGE_NAMES[args.storage]
    n = args.n
    n_side = 8
    t0 = time.perf_counter()
    if args.workload == "sphere32":
        n = 32
        log("generating sphere scene 32^3, 8 cameras 128x128")
        sc = scenes.sphere_scene()
    else:
        log(f"generating terrain scene n={n}, {n_side * n_side} cameras 1024x1024")
        sc = scenes.terrain_scene(n=n, n_side=n_side, W=1024, H=1024, f=1536.0, device="cuda")
    log(f"scene ready in {time.perf_counter() - t0:.1f} s")
    H, W = sc.depth.shape[1:]
    depth = torch.from_numpy(sc.depth).to(dev)
    ctx = tgv.Context(0)
    g = tgv.grid_from(sc.grid)
    bins = tgv.Bins()
    nvox = g.nx * g.ny * g.nz
    if args.schedule == "auto":
        # the library's default for a block with no tile given
        args.schedule = "fused2" if nvox * fused_bytes_per_voxel(storage) > (48 << 20) else "fused"
    sched = tgv.SCHED_FUSED2 if args.schedule == "fused2" else tgv.SCHED_FUSED
    params = tgv.Params(iters=args.iters, storage=storage, schedule=sched)
    pyr = torch.empty((len(sc.cams), ctx.pyramid_floats(W, H)), dtype=torch.float32, device=dev)
    hist = torch.empty((nvox, 8), dtype=torch.int16, device=dev)
    u = torch.empty(nvox, dtype=torch.float32, device=dev)
    cams = tgv.cameras_from(sc.cams)

    def step():
        ctx.build_pyramids(depth, out=pyr)
        ctx.build_histograms(pyr, W, H, cams, g, bins, out=hist)
        u.zero_()
        return ctx.solve(g, hist, u, params, bins, stats=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    stats = None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        stats = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps
    updates = nvox * args.iters
    value = updates * args.steps / elapsed
    log(f"{args.steps} steps in {elapsed:.3f} s; gap_rel {stats['gap_rel']:.3g}, nonfinite {stats['nonfinite']}")

    # phase split and the fused kernel's average duration (HIP events on the
    # stream the library launches on)
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(s)
    ctx.build_pyramids(depth, out=pyr)
    ev[1].record(s)
    ctx.build_histograms(pyr, W, H, cams, g, bins, out=hist)
    ev[2].record(s)
    torch.cuda.synchronize()
    pyr_ms, hist_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    pairs = nvox * len(sc.cams)  # voxel x camera pairs before the cull
    # VALU ceiling of the histogram kernel: its measured VALU instructions
    # (SQ_INSTS_VALU of this workload's launch, committed counter summary)
    # issued at one wave64 instruction per SIMD per two cycles (the 157.3
    # TFLOP/s FP32 vector peak: 32 lanes per SIMD per cycle) on 1024 SIMDs
    hist_rate = dict(pairs=pairs, ms=hist_ms, pairs_per_s=pairs / (hist_ms * 1e-3))
    vi = hist_valu_instructions() if n == 256 and len(sc.cams) == 64 else None
    if vi is not None:
        floor_ms = vi / (1024 * 2.4e9 * 0.5) * 1e3
        hist_rate.update(valu_wave_instructions=vi, lane_instructions_per_pair=round(vi * 64 / pairs, 1),
                         valu_floor_ms=round(floor_ms, 4), frac_of_valu_ceiling=round(floor_ms / hist_ms, 3),
                         valu_source="profiles/k_hist_terrain256_counters.md (SQ_INSTS_VALU)")
    def kernel_roofline(schedule):
        """Average launch time of the schedule's dominant kernel (HIP events on
        the library's stream: median difference of 400- and 200-iteration
        solves) against its algorithmic bytes per launch."""
        sch = tgv.SCHED_FUSED2 if schedule == "fused2" else tgv.SCHED_FUSED
        it_hi, it_lo = (400, 200) if n >= 128 else (2000, 1000)
        times = {}
        for its in (it_lo, it_hi) * 5:
            u.zero_()
            p2 = tgv.Params(iters=its, storage=storage, schedule=sch)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            ctx.solve(g, hist, u, p2, bins)
            e1.record(s)
            torch.cuda.synchronize()
            times.setdefault(its, []).append(e0.elapsed_time(e1))
        # one launch of the dominant kernel: one iteration (fused) or two (fused2)
        per_launch = 2 if schedule == "fused2" else 1
        k_ms = (float(np.median(times[it_hi])) - float(np.median(times[it_lo]))) / (it_hi - it_lo) * per_launch
        bpu = bytes_per_update(storage)
        achieved = bpu * per_launch * nvox / (k_ms * 1e-3) / 1e9
        bpv = fused_bytes_per_voxel(storage)
        one_pass = bpv * nvox / (k_ms * 1e-3) / 1e9
        if schedule == "fused2":
            tile = f"{params.tile_y or 7}x{params.tile_z or 'auto'}"
        else:
            big = nvox * fused_bytes_per_voxel(storage) > (256 << 20)
            tile = f"{params.tile_y or (8 if storage == 0 and big else 4)}x{params.tile_z or 32}"
        traffic = measured_traffic(storage, tile, schedule) if n == 256 else None
        log(f"{schedule} launch {k_ms * 1e3:.1f} us ({per_launch} iteration(s)) -> {achieved:.0f} GB/s at "
            f"{bpu} B per update, {one_pass:.0f} GB/s at the pass's {bpv} B per voxel")
        return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, tile=tile,
                    kernel=("tgv fused iteration" if per_launch == 1 else "tgv two fused iterations per pass"),
                    basis=f"{bpu} B per voxel-update (plain fused step: read u, ubar, v, vbar, p, q, histogram; "
                          f"write u, ubar, v, vbar, p, q) x {per_launch} update(s) per voxel per launch x "
                          f"{nvox} voxels / average launch time",
                    bytes_per_update=bpu, voxels_per_launch=nvox, iterations_per_launch=per_launch,
                    avg_launch_ms=round(k_ms, 5), us_per_iteration=round(1e3 * k_ms / per_launch, 2),
                    one_pass_basis=dict(bytes_per_voxel_per_launch=bpv, achieved=round(one_pass, 1),
                                        frac=round(one_pass / HBM_PEAK_GBS, 4),
                                        note="the bytes the launch's single pass must move: read u, v, p, q, "
                                             "histogram; write u, v, p, q"),
                    measured_traffic=(None if traffic is None else dict(
                        bytes_per_launch=traffic, GBs=round(traffic / (k_ms * 1e-3) / 1e9, 1),
                        frac=round(traffic / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        source="rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size")))

    def copy_ceiling():
        """HBM rate of a plain streaming copy on this GPU (1 GiB read + 1 GiB
        written): the library's copy kernel in each of its 32 shapes (16-byte
        vectors per lane, non-temporal or not, workgroups per CU), median of 3
        each, the best one reported; torch's device copy beside it."""
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        nbytes = 2 * (1 << 30)

        def med_ms(fn, reps):
            ms = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                fn()
                e1.record(s)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            return float(np.median(ms))

        per = {}
        for var in range(32):
            ctx.stream_copy(a, b, var)
            per[var] = med_ms(lambda: ctx.stream_copy(a, b, var), 3)
        best = min(per, key=per.get)
        b.zero_()
        ctx.stream_copy(a, b, best)
        torch.cuda.synchronize()
        assert torch.equal(a, b), "stream copy result differs"
        b.copy_(a)
        t_torch = med_ms(lambda: b.copy_(a), 5)
        del a, b
        t = per[best]
        return dict(GBs=round(nbytes / (t * 1e-3) / 1e9, 1), bytes=nbytes, ms=round(t, 4),
                    kernel=f"tgv_stream_copy variant {best} (vectors per lane {1 << (best & 3)}, "
                           f"{'non-temporal' if best & 4 else 'cached'}, {2 << ((best >> 3) & 3)} workgroups per CU), "
                           "best of 32 shapes, median of 3",
                    worst_shape_GBs=round(nbytes / (max(per.values()) * 1e-3) / 1e9, 1),
                    torch_copy_GBs=round(nbytes / (t_torch * 1e-3) / 1e9, 1))

    roof = None
    reference = None
    copy = None
    if not args.kernel_only:
        roof = kernel_roofline(args.schedule)
        if args.schedule == "fused2":
            # the one-iteration kernel on the same block, for comparison
            reference = kernel_roofline("fused")
        copy = copy_ceiling()
        log(f"plain copy: {copy['GBs']:.0f} GB/s (torch's copy {copy['torch_copy_GBs']:.0f} GB/s)")

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        cpu = cpu_baseline(sc, bins.centers32(), crop=min(96, n), iters_sample=200 if n >= 64 else 600)
        cpu.pop("hist_pairs_per_s", None)

    lat_ms = sorted(1000.0 * x for x in lat)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if storage == 0 else ("f32 compute, " + args.storage + " storage"),
        "data": "synthetic",
        "config": {"workload": args.workload if args.workload != "terrain256" else f"terrain{n}",
                   "grid": [g.nx, g.ny, g.nz], "cameras": len(sc.cams),
                   "image": [W, H], "iters": args.iters, "bins": 7, "storage": args.storage,
                   "schedule": args.schedule,
                   "step": "pyramids + cull + histograms + init + iterations + gap"},
        "roofline": roof,
        "one_pass_kernel": reference,
        "copy_ceiling": copy,
        "cpu_baseline": cpu,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "phases_ms": {"pyramids": pyr_ms, "histograms": hist_ms},
        "histograms": hist_rate,
        "gap_rel": stats["gap_rel"],
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


def bench_city_batch(args):
    """512 octree-leaf-like blocks of the city (edges log-uniform 32..128 plus a
    2-voxel halo), 500 iterations each: one batched solve (a persistent
    launch per two iterations over all blocks, graph replay) against the
    batched one-iteration kernel with autotuned tiles and against solving
    the blocks one by one with the library's defaults; results compared bit
    for bit."""
    import torch
    import paper_2107_14790_amd as tgv
    from paper_2107_14790_amd.autotune import Autotuner
    import scenes

    iters = args.iters or 500
    storage = tgv.STORAGE_NAMES[args.storage]
    if not os.path.exists(scenes._RAYLIB):
        scenes.build_raycaster()
    t0 = time.perf_counter()
    sc, hf = scenes.city_scene(device="cuda")
    log(f"city scene: {len(sc.cams)} cameras 1024x1024 in {time.perf_counter() - t0:.1f} s")
    grids = scenes.city_blocks(sc, n_blocks=args.blocks)
    ctx = tgv.Context(0)
    H, W = sc.depth.shape[1:]
    depth = torch.from_numpy(sc.depth).cuda()
    cams = tgv.cameras_from(sc.cams)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    pyr = ctx.build_pyramids(depth)
    e1.record(s)
    torch.cuda.synchronize()
    pyr_ms = e0.elapsed_time(e1)
    del depth
    hists, states, u0s = [], [], []
    interior = padded = 0
    e0.record(s)
    for g in grids:
        gc = tgv.grid_from(g)
        hists.append(ctx.build_histograms(pyr, W, H, cams, gc))
        nvox = gc.nx * gc.ny * gc.nz
        padded += nvox
        interior += (gc.nx - 2 * gc.halo) * (gc.ny - 2 * gc.halo) * (gc.nz - 2 * gc.halo)
        states.append(tgv.State(ctx, gc, storage))
        u0s.append(torch.zeros(nvox, device="cuda"))
    e1.record(s)
    torch.cuda.synchronize()
    hist_ms = e0.elapsed_time(e1)
    log(f"{len(grids)} blocks: {padded / 1e6:.1f} M padded voxels, histograms {hist_ms:.0f} ms")
    t0 = time.perf_counter()
    tuner = Autotuner(ctx)
    tune = tuner.tune(grids, storage)
    one = tune["by_schedule"]["fused"]
    log(f"autotune {time.perf_counter() - t0:.1f} s: {tune['schedule']} tile_y {tune['tile_y']}, classes "
        + ", ".join(f"{k}:{v['best']}" for k, v in tune["classes"].items())
        + f"; checked on the batch: {tune['checked_on_batch']}")
    # the autotuner's pick (the headline); the library's default batched
    # schedule (two iterations per launch, 64 x 7 tiles, chunks of up to 32
    # planes); the best one-iteration-per-launch shapes; blocks one by one
    # with the library's defaults
    p_tuned = Autotuner.params(tune, iters, storage, flags=tgv.FLAG_GRAPH)
    p_default = tgv.Params(iters=iters, storage=storage, schedule=tgv.SCHED_FUSED2, flags=tgv.FLAG_GRAPH)
    p_one = tgv.Params(iters=iters, storage=storage, tile_y=one["tile_y"], schedule=tgv.SCHED_FUSED,
                       flags=tgv.FLAG_GRAPH)

    def batched():
        for st, u0 in zip(states, u0s):
            st.reset(u0)
        ctx.solve_batch(states, hists, p_tuned, tile_z=tune["tile_z"])

    def batched_default():
        for st, u0 in zip(states, u0s):
            st.reset(u0)
        ctx.solve_batch(states, hists, p_default)

    def batched_one_pass():
        for st, u0 in zip(states, u0s):
            st.reset(u0)
        ctx.solve_batch(states, hists, p_one, tile_z=one["tile_z"])

    def plain_default():
        # one by one with the library's defaults (schedule AUTO, tiles and chunk depth chosen per block)
        for st, u0, h in zip(states, u0s, hists):
            st.reset(u0)
            ctx.solve(st.grid, h, None, tgv.Params(iters=iters, storage=storage), state=st)

    batched()  # warm (graph capture)
    torch.cuda.synchronize()
    times = {}
    for name, fn in (("batched", batched), ("batched_default", batched_default),
                     ("batched_one_pass", batched_one_pass), ("plain_default", plain_default)):
        ts = []
        for _ in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        times[name] = ts
        log(f"{name}: {[round(x, 3) for x in ts]} s")
        if name == "batched":
            ref = [st.export()["u"] for st in states[:8]]
        if name == "plain_default":
            same_default = all(torch.equal(a, st.export()["u"]) for a, st in zip(ref, states[:8]))
        if name == "batched_one_pass":
            same_one = all(torch.equal(a, st.export()["u"]) for a, st in zip(ref, states[:8]))
        if name == "batched_default":
            same_bd = all(torch.equal(a, st.export()["u"]) for a, st in zip(ref, states[:8]))
    tb, tp = min(times["batched"]), min(times["plain_default"])
    bpv = bytes_per_update(storage)
    out = {
        "metric": METRIC,
        "value": interior * iters / tb,
        "unit": "voxel-updates/s",
        "n_gpus": 1, "steps": len(times["batched"]), "warmup": 1,
        "ms_per_step": 1000 * tb,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if storage == 0 else "f32 compute, " + args.storage + " storage",
        "data": "synthetic",
        "config": {"workload": "city_batch", "blocks": len(grids), "edge": "log-uniform 32..128 + 2 halo",
                   "iters": iters, "cameras": len(sc.cams), "image": [W, H], "padded_voxels": padded,
                   "interior_voxels": interior, "tuned": {"schedule": tune["schedule"], "tile_y": tune["tile_y"],
                                                          "classes": tune["classes"],
                                                          "checked_on_batch": tune["checked_on_batch"]}},
        "batched": {"s": tb, "blocks_per_s": len(grids) / tb, "updates_per_s_interior": interior * iters / tb,
                    "algorithmic_GBs": bpv * padded * iters / tb / 1e9,
                    "shapes": "autotuned (schedule, tile_y, per-block tile_z)"},
        "batched_library_default": {"s": min(times["batched_default"]),
                                    "updates_per_s_interior": interior * iters / min(times["batched_default"]),
                                    "shapes": "two iterations per launch, 64 x 7 tiles, chunks of up to 32 planes"},
        "batched_one_pass_autotuned": {"s": min(times["batched_one_pass"]), "tile_y": one["tile_y"],
                                       "updates_per_s_interior": interior * iters / min(times["batched_one_pass"])},
        "plain_library_defaults": {"s": min(times["plain_default"]),
                                   "blocks_per_s": len(grids) / min(times["plain_default"]),
                                   "updates_per_s_interior": interior * iters / min(times["plain_default"])},
        "speedup_batched_vs_plain": tp / tb,
        "plain": "blocks one by one with the library's defaults (plain_library_defaults)",
        "bitwise_same_alone_and_batched": bool(same_default and same_one and same_bd),
        "phases_ms": {"pyramids": pyr_ms, "histograms_all_blocks": hist_ms},
    }
    print(json.dumps(out), flush=True)


def bench_city_serve(args):
    """A Poisson stream of block solves (edges log-uniform 32..192 plus a
    2-voxel halo) from the city: histograms built on arrival from resident
    pyramids, states resident in HBM under a 200 GB admission budget,
    continuous batching in ticks of 50 iterations, 500 iterations per block.
    Reported at the configured rate (above capacity: queueing dominates the
    latency) and at 0.5, 0.8 and 0.95 of the service rate measured there."""
    import torch
    import paper_2107_14790_amd as tgv
    from paper_2107_14790_amd.serve import GpuBackend, Request, Server, latency_stats, poisson_arrivals
    import scenes

    iters = args.iters or 500
    storage = tgv.STORAGE_NAMES[args.storage]
    if not os.path.exists(scenes._RAYLIB):
        scenes.build_raycaster()
    t0 = time.perf_counter()
    sc, hf = scenes.city_scene(device="cuda")
    log(f"city scene in {time.perf_counter() - t0:.1f} s")
    ctx = tgv.Context(0)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    torch.cuda.synchronize()
    pool = scenes.city_blocks(sc, n_blocks=max(args.arrivals, 64), e_min=32, e_max=192, seed=5)
    if args.schedule == "fused2":  # two iterations per persistent launch
        params = tgv.Params(iters=iters, storage=storage, schedule=tgv.SCHED_FUSED2, flags=tgv.FLAG_GRAPH)
    else:
        params = tgv.Params(iters=iters, storage=storage, schedule=tgv.SCHED_FUSED, tile_y=4, flags=tgv.FLAG_GRAPH)
    budget = 200 << 30

    def run(rate, count, seed):
        t = poisson_arrivals(rate, count, seed)
        reqs = [Request(i, pool[i % len(pool)], float(t[i]), iters) for i in range(count)]
        be = GpuBackend(ctx, pyr, W, H, sc.cams, params=params, keep_outputs=False)
        srv = Server(be, budget, tick_iters=50)
        t1 = time.perf_counter()
        res = srv.run(reqs)
        wall = time.perf_counter() - t1
        st = latency_stats(res)
        vox = sum(int(np.prod(r.grid.n)) for r in reqs)
        interior = sum(int(np.prod([v - 2 * r.grid.halo for v in r.grid.n])) for r in reqs)
        st.update(rate=rate, arrivals=count, wall_s=wall, blocks_per_s=st["n_ok"] / wall,
                  updates_per_s_interior=interior * iters / wall, updates_per_s_padded=vox * iters / wall,
                  ticks=srv.ticks, max_active=srv.max_active_seen, peak_resident_GB=srv.peak_used / 2 ** 30)
        log(f"rate {rate:.1f}/s: p50 {st.get('p50_s', 0):.2f} s p99 {st.get('p99_s', 0):.2f} s, "
            f"{st['blocks_per_s']:.1f} blocks/s, max active {srv.max_active_seen}")
        return st, res

    run(200.0, 8, 99)  # warm (graph capture, allocator)
    hot, _ = run(args.rate, args.arrivals, 5)
    cap = hot["blocks_per_s"]
    # below capacity: Poisson arrivals at fractions of the measured service rate
    below = {}
    for k, frac in enumerate((0.5, 0.8, 0.95)):
        below[str(frac)], _ = run(frac * cap, max(24, args.arrivals // 5), 6 + k)
    # alone vs in the mix: re-serve a few blocks alone and compare checksums
    be = GpuBackend(ctx, pyr, W, H, sc.cams, params=params, keep_outputs=False)
    mix_reqs = [Request(i, pool[i], 0.0, iters) for i in range(6)]
    mix = Server(be, budget, tick_iters=50).run(mix_reqs)
    alone = [Server(be, budget, tick_iters=50).run([Request(0, pool[i], 0.0, iters)])[0] for i in range(6)]
    same = all(float(a.output) == float(m.output) for a, m in zip(alone, mix))
    out = {
        "metric": METRIC,
        "value": hot["updates_per_s_interior"],
        "unit": "voxel-updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1000 * hot["wall_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if storage == 0 else "f32 compute, " + args.storage + " storage",
        "data": "synthetic",
        "config": {"workload": "city_serve", "rate_per_s": args.rate, "arrivals": args.arrivals,
                   "edge": "log-uniform 32..192 + 2 halo", "iters": iters, "budget_GB": 200, "tick_iters": 50,
                   "schedule": args.schedule},
        "latency_s": {"p50": hot.get("p50_s"), "p99": hot.get("p99_s")},
        "at_rate": hot,
        "measured_capacity_blocks_per_s": cap,
        "at_capacity_fraction": below,
        "bitwise_same_alone_and_mixed": bool(same),
    }
    print(json.dumps(out), flush=True)


def zero_crossing_errors(u, ref, shape):
    """Zero-crossing comparison of two fields on a block (torch tensors,
    same shape): on every grid edge where both fields change sign, the
    crossing position t = u_a / (u_a - u_b) (in voxels) of u against ref;
    plus the fraction of edges whose sign change differs and the largest
    |u - ref| where |ref| < 0.5."""
    import torch
    nx, ny, nz = shape
    a = u.double().reshape(nz, ny, nx)
    b = ref.double().reshape(nz, ny, nx)
    errs, diff, tot = [], 0, 0
    for ax in range(3):
        a0, a1 = a.narrow(ax, 0, a.shape[ax] - 1), a.narrow(ax, 1, a.shape[ax] - 1)
        b0, b1 = b.narrow(ax, 0, b.shape[ax] - 1), b.narrow(ax, 1, b.shape[ax] - 1)
        sa = (a0 > 0) != (a1 > 0)
        sb = (b0 > 0) != (b1 > 0)
        both = sa & sb
        ta = a0[both] / (a0[both] - a1[both])
        tb = b0[both] / (b0[both] - b1[both])
        errs.append((ta - tb).abs())
        diff += int((sa != sb).sum().item())
        tot += int(sb.sum().item())
    e = torch.cat(errs)
    near = b.abs() < 0.5
    return {"zc_max_vox": float(e.max().item()) if e.numel() else 0.0,
            "zc_mean_vox": float(e.mean().item()) if e.numel() else 0.0,
            "zc_edges": int(e.numel()), "sign_pattern_diff_frac": diff / max(tot, 1),
            "max_abs_near_surface": float((a - b).abs()[near].max().item()) if near.any() else 0.0}


def bench_city_precision(args):
    """One 384^3 block of the city fusing 256 depth maps of 2048^2, 1000
    iterations, with v, p, q stored in float32, float16 and bfloat16 (float32
    arithmetic and u): time per iteration, bandwidth gain and zero-crossing
    error against the float32-storage solve; and all three against the
    float64 oracle on the whole block (histograms bit for bit, then u after
    the same iterations: max |u - u_oracle| and the zero crossings)."""
    import torch
    import oracle
    import paper_2107_14790_amd as tgv
    import scenes

    iters = args.iters or 1000
    n = args.n if args.n != 256 else 384
    sched = tgv.SCHED_FUSED2 if args.schedule == "fused2" else tgv.SCHED_FUSED
    if not os.path.exists(scenes._RAYLIB):
        scenes.build_raycaster()
    t0 = time.perf_counter()
    sc, hf = scenes.city_scene(W=2048, H=2048, f=2048.0, sigma=0.3 / 2048, device="cuda")
    log(f"city scene 256 x 2048^2 in {time.perf_counter() - t0:.1f} s")
    h = float(np.float32(0.4 / n))
    centre = np.array([0.5, 0.5, 0.6])
    grid = scenes.Grid((centre - 0.5 * n * h).astype(np.float32), h, (n, n, n), 0)
    ctx = tgv.Context(0)
    H, W = sc.depth.shape[1:]
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    g = tgv.grid_from(grid)
    hist = ctx.build_histograms(pyr, W, H, sc.cams, g)
    torch.cuda.synchronize()
    nvox = n ** 3
    s = torch.cuda.current_stream()
    res, us = {}, {}
    for name in ("f32", "f16", "bf16"):
        st = tgv.STORAGE_NAMES[name]
        u = torch.zeros(nvox, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.solve(g, hist, u, tgv.Params(iters=5, storage=st, schedule=sched))  # warm
        u.zero_()
        e0.record(s)
        stats = ctx.solve(g, hist, u, tgv.Params(iters=iters, storage=st, schedule=sched))
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        us[name] = u.clone()
        bpv = bytes_per_update(st)
        res[name] = {"s": ms / 1e3, "us_per_iter": 1e3 * ms / iters, "updates_per_s": nvox * iters / (ms / 1e3),
                     "algorithmic_GBs": bpv * nvox * iters / (ms / 1e3) / 1e9, "bytes_per_update": bpv,
                     "frac_of_peak": bpv * nvox * iters / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
        log(f"{name}: {ms / 1e3:.2f} s, {1e3 * ms / iters:.1f} us/iter")
        del u
    for name in ("f16", "bf16"):
        res[name]["speedup_vs_f32"] = res["f32"]["s"] / res[name]["s"]
        res[name]["vs_f32_gpu"] = zero_crossing_errors(us[name], us["f32"], (n, n, n))
    # the float64 oracle on the whole block, on the host's cores (its per-voxel
    # loops split over threads: bit for bit its serial result), in chunks so
    # that progress is visible
    vs_oracle = None
    if not args.no_oracle:
        k = max(1, min(16, os.cpu_count() or 1))
        t0 = time.perf_counter()
        opyr = oracle.pyramids(sc.depth)
        osc = scenes.Scene(None, sc.cams, grid)
        href = np.empty((nvox, 8), dtype=np.uint16)
        plane = n * n
        with oracle.threads(k):
            for z0 in range(0, n, 32):
                vox = np.arange(z0 * plane, min(n, z0 + 32) * plane, dtype=np.int64)
                href[vox], _ = oracle.histograms(osc, opyr, vox=vox)
                log(f"oracle histograms to plane {min(n, z0 + 32)} of {n} ({time.perf_counter() - t0:.0f} s)")
        del opyr
        hist_same = bool(np.array_equal(hist.cpu().numpy().view(np.uint16), href))
        log(f"whole-block histograms bit-exact against the oracle: {hist_same}")
        ost = None
        chunk = 100
        with oracle.threads(k):
            for done in range(0, iters, chunk):
                step = min(chunk, iters - done)
                ost = oracle.solve(href, (n, n, n), scenes.default_bins(), step, state=ost)
                log(f"oracle {done + step}/{iters} iterations ({time.perf_counter() - t0:.0f} s)")
        uref = torch.from_numpy(ost.u).cuda()
        del ost, href
        vs_oracle = {"threads": k, "oracle_s": time.perf_counter() - t0, "histograms_bit_exact": hist_same}
        for name in ("f32", "f16", "bf16"):
            vs_oracle[name] = zero_crossing_errors(us[name], uref, (n, n, n))
            d = (us[name].double() - uref).abs()
            vs_oracle[name]["max_abs"] = float(d.max().item())
            vs_oracle[name]["mean_abs"] = float(d.mean().item())
            log(f"{name} vs float64 oracle: max |u - u_ref| {vs_oracle[name]['max_abs']:.3g}, zero crossings "
                f"max {vs_oracle[name]['zc_max_vox']:.3g} mean {vs_oracle[name]['zc_mean_vox']:.3g} voxel")
    out = {
        "metric": METRIC,
        "value": res["f16"]["updates_per_s"],
        "unit": "voxel-updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * res["f16"]["s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 compute, f16 storage (value); f32 and bf16 storage reported beside",
        "data": "synthetic",
        "config": {"workload": "city_precision", "grid": [n, n, n], "cameras": len(sc.cams), "image": [W, H],
                   "iters": iters, "h": h, "schedule": args.schedule},
        "storage": res,
        "vs_float64_oracle": vs_oracle,
    }
    print(json.dumps(out), flush=True)


def bench_next(args):
    """The rows that widen the core path, measured on the benchmark's 256^3
    terrain block (64 nadir 1024^2 depth maps): coarse-to-fine (3 levels x
    200 iterations) beside the plain 1000-iteration solve; the TV-L1 model
    (Eq. 1) for 1000 iterations; the histogram build with four terrestrial
    360-degree scans (equirectangular 4096 x 2048, vote 5) fused with the
    stereo maps in one call; and the zero-level extraction from the solved
    block."""
    import math
    import torch
    import paper_2107_14790_amd as tgv
    import scenes

    n = args.n
    iters = args.iters or 1000
    t0 = time.perf_counter()
    sc = scenes.terrain_scene(n=n, n_side=8, W=1024, H=1024, f=1536.0, device="cuda")
    sd, scams = scenes.terrain_scans360(n=n, device="cuda")
    log(f"terrain {n}^3 with {len(sc.cams)} stereo maps and {len(scams)} 360-degree scans "
        f"({sd.shape[2]}x{sd.shape[1]}) in {time.perf_counter() - t0:.1f} s")
    ctx = tgv.Context(0)
    H, W = sc.depth.shape[1:]
    g = tgv.grid_from(sc.grid)
    nvox = n ** 3
    s = torch.cuda.current_stream()
    pyr = ctx.build_pyramids(torch.from_numpy(sc.depth).cuda())
    hist = ctx.build_histograms(pyr, W, H, sc.cams, g)
    torch.cuda.synchronize()

    def timed(fn, reps=3):
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    def per_iteration_ms(params_of):
        # median difference of 400- and 200-iteration solves
        u = torch.zeros(nvox, device="cuda")
        t = {}
        for its in (200, 400) * 3:
            u.zero_()
            t.setdefault(its, []).append(timed(lambda: ctx.solve(g, hist, u, params_of(its)), reps=1))
        return (float(np.median(t[400])) - float(np.median(t[200]))) / 200

    out = {}
    # plain solve, the reference of the rows below
    u = torch.zeros(nvox, device="cuda")
    ms_plain = timed(lambda: (u.zero_(), ctx.solve(g, hist, u, tgv.Params(iters=iters))))
    u_plain = u.clone()
    # 1. coarse-to-fine
    levels, it_lvl = 3, 200
    c2f_updates = sum(math.ceil(n / 2 ** k) ** 3 for k in range(levels)) * it_lvl
    ms_c2f = timed(lambda: ctx.solve_coarse_to_fine(pyr, W, H, sc.cams, g, levels, tgv.Params(iters=it_lvl)))
    out["coarse_to_fine"] = {"levels": levels, "iters_per_level": it_lvl, "ms": ms_c2f,
                             "updates_per_s": c2f_updates / (ms_c2f * 1e-3),
                             "plain_solve_ms": ms_plain, "plain_iters": iters,
                             "note": "histograms of every level built inside the call; includes them"}
    log(f"coarse-to-fine {levels} x {it_lvl}: {ms_c2f:.1f} ms (plain {iters}: {ms_plain:.1f} ms)")
    # 2. TV-L1: whole solve and the dominant kernel's per-iteration time
    ms_tv = timed(lambda: (u.zero_(), ctx.solve(g, hist, u, tgv.Params(iters=iters, flags=tgv.FLAG_TVL1))))
    it_tv = per_iteration_ms(lambda its: tgv.Params(iters=its, flags=tgv.FLAG_TVL1))
    it_tgv = per_iteration_ms(lambda its: tgv.Params(iters=its))
    # The plain TV-L1 step reads u, ubar, p(3) and the histogram and writes u,
    # ubar and p: 56 B per update.  The rotated pass needs 48 B per voxel (u,
    # p, histogram in; u, p out), and the two-iteration kernel (the default
    # on this block) makes one pass per two iterations and moves no v or q.
    tv_launch_ms = 2 * it_tv
    tv_bpu = 56
    out["tvl1"] = {"iters": iters, "ms": ms_tv, "updates_per_s": nvox * iters / (ms_tv * 1e-3),
                   "us_per_iteration": 1e3 * it_tv, "tgv_us_per_iteration": 1e3 * it_tgv,
                   "roofline": {"bound": "hbm", "kernel": "tgv two fused iterations per pass (TV-L1)",
                                "achieved": round(tv_bpu * 2 * nvox / (tv_launch_ms * 1e-3) / 1e9, 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(tv_bpu * 2 * nvox / (tv_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                "bytes_per_update": tv_bpu, "iterations_per_launch": 2,
                                "avg_launch_ms": round(tv_launch_ms, 5),
                                "one_pass_basis": {"bytes_per_voxel_per_launch": 48,
                                                   "achieved": round(48 * nvox / (tv_launch_ms * 1e-3) / 1e9, 1),
                                                   "frac": round(48 * nvox / (tv_launch_ms * 1e-3) / 1e9
                                                                 / HBM_PEAK_GBS, 4)}}}
    log(f"TV-L1 {iters}: {ms_tv:.1f} ms, {1e3 * it_tv:.1f} us per iteration (TGV {1e3 * it_tgv:.1f})")
    # 3. vote 5: stereo maps plus terrestrial 360-degree scans at their own
    # resolution, one histogram call over both
    cams_all = scenes.concat_cameras(sc.cams, scams)
    pyr_all, offs_all = ctx.build_pyramids_mixed([torch.from_numpy(sc.depth).cuda(), torch.from_numpy(sd).cuda()])
    h_all = ctx.build_histograms_ex(pyr_all, offs_all, cams_all, g)
    ms_h = timed(lambda: ctx.build_histograms_ex(pyr_all, offs_all, cams_all, g, out=h_all), reps=5)
    ms_h0 = timed(lambda: ctx.build_histograms(pyr, W, H, sc.cams, g, out=hist), reps=5)
    pairs = nvox * len(cams_all)
    out["vote5_scans"] = {"stereo_maps": len(sc.cams), "stereo_image": [W, H], "scans": len(scams),
                          "scan_image": [int(sd.shape[2]), int(sd.shape[1])], "ms": ms_h,
                          "pairs_per_s": pairs / (ms_h * 1e-3), "stereo_only_ms": ms_h0,
                          "scan_pairs_per_s": nvox * len(scams) / ((ms_h - ms_h0) * 1e-3),
                          "max_count": int(h_all.view(torch.int16).to(torch.int32).max().item())}
    del pyr_all
    log(f"histograms with scans: {ms_h:.2f} ms for {len(cams_all)} maps (stereo only {ms_h0:.2f} ms)")
    # 4. zero level of the solved block: one call into a preallocated
    # output (count, offsets, write; the call synchronises)
    cnt = ctx.extract_crossings(g, u_plain).shape[0]
    pts = torch.empty((cnt, 4), dtype=torch.float32, device="cuda")
    ms_x = timed(lambda: ctx.extract_crossings(g, u_plain, out=pts), reps=5)
    ms_x2 = timed(lambda: ctx.extract_crossings(g, u_plain), reps=5)
    # two passes over u (count, write) plus 16 B per point
    xbytes = 2 * 4 * nvox + 16 * cnt
    out["zero_level"] = {"points": cnt, "ms": ms_x, "voxels_per_s": nvox / (ms_x * 1e-3),
                         "ms_count_then_write": ms_x2,
                         "note": "one call into a preallocated output, including its host synchronisation",
                         "roofline": {"bound": "hbm", "achieved": round(xbytes / (ms_x * 1e-3) / 1e9, 1),
                                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": round(xbytes / (ms_x * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                      "bytes": xbytes}}
    log(f"zero level: {cnt} points in {ms_x:.2f} ms")
    res = {
        "metric": METRIC,
        "value": nvox * iters / (ms_tv * 1e-3),
        "unit": "voxel-updates/s",
        "n_gpus": 1, "steps": 3, "warmup": 1,
        "ms_per_step": ms_tv,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "next", "grid": [n, n, n], "cameras": len(sc.cams), "image": [W, H],
                   "iters": iters, "value_is": "TV-L1 updates/s"},
    }
    res.update(out)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
