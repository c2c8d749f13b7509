#!/usr/bin/env python3
"""Throughput of chunked-SVDAG primary-ray traversal on one MI355X.

One step = one view through the whole hot path: the chunk stage (LOD pick
and frustum cull per chunk) and the per-pixel trace (chunk walk, DAG
traversal, material resolve, record write), with every chunk DAG already
resident in HBM.  Steps cycle over 10 seeded camera poses.

Prints one JSON line (rank 0).  Besides the throughput it reports:
  roofline      for the trace kernel: algorithmic bytes per launch (mean
                bytes per ray from the oracle's visit counts x rays) over the
                kernel's mean duration over the timed steps (HIP events
                stamped by its own dispatches on its stream), against
                the 8 TB/s HBM peak; beside it the no-reuse bound (every read
                a 64-B sector), the compulsory bytes (each touched byte once,
                from the oracle's touch count) and the HBM traffic the
                counters measured;
  valu_issue    the trace kernel's VALU instructions (counters) per second
                against the issue peak, and its lane utilisation;
  cpu_baseline  the CPU oracle timed on a bounded sample of the same views.

Other workloads: --workload terrain1024 | noise64 | map1024.  map1024 (32x32
chunks of 1024^3) is generated on the GPU with --gen gpu (the same bytes as
the host generator) and runs with --no-cpu-baseline, since the oracle cannot
build all of its chunks within the run.  The default run also times the
per-view leg of terrain1024 and noise64 (other_workloads; --other-workloads).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (scene kind, lod_count, thresholds, description)
    "map512": ("map512", 4, (256, 1024, 4096),
               "map512: 16x16x1 chunks of 512^3 (8192x8192x512) terrain+caves+boxes, 4 LODs, "
               "frustum culling, 2560x1440 rays, 10 seeded views"),
    "map1024": ("map1024", 4, (256, 1024, 4096),
                "map1024: 32x32x1 chunks of 1024^3 (32768x32768x1024) terrain+caves+boxes, 4 LODs, "
                "frustum culling, 2560x1440 rays, 10 seeded views"),
    "terrain1024": ("terrain1024", 1, (256, 1024, 4096),
                    "terrain1024: one 1024^3 terrain chunk with caves, 1920x1080 rays, 10 seeded views"),
    "noise64": ("noise64", 1, (256, 1024, 4096),
                "noise64: one 64^3 value-noise chunk (~30% fill), 256x256 rays, 10 seeded views"),
}
HBM_PEAK_GBS = 8000.0
METRIC = "primary rays/s (Grays/s) of SVDAG traversal at 1440p; p50/p99 view latency under load"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def default_tune_cache():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_2505_02017_amd", "tune.txt")


def tune_cache_path(args):
    """The tuning cache file (its directory created), or None (no cache, or
    a directory that cannot be created)."""
    if not args.tune_cache or args.tune_cache == "none":
        return None
    try:
        os.makedirs(os.path.dirname(os.path.abspath(args.tune_cache)), exist_ok=True)
    except OSError as e:
        log(f"tuning cache disabled: {e}")
        return None
    return args.tune_cache


def tune_world(svdag, world, frames, out, flags, cache, stream):
    """svd_world_tune through the cache; a cache that cannot be written
    leaves the tuned choice applied (the library's contract) and is
    reported, not fatal."""
    try:
        return svdag.svd_world_tune(world, frames, out, flags, reps=3, cache_path=cache, stream=stream), cache
    except svdag.SvdError as e:
        if e.code != svdag.SVD_EIO:
            raise
        log(f"tuning cache not written ({e}); tuning without it")
        return svdag.svd_world_tune(world, frames, out, flags, reps=3, cache_path=None, stream=stream), None


def counter_profile(workload):
    """Counter-derived figures of the trace kernel from the committed profile
    (profiles/trace_kernel_<workload>_traffic.txt), or {} if that profile was
    taken on a different kernel source than the one built here."""
    from paper_2505_02017_amd.build import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"trace_kernel_{workload}_traffic.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.split()[0] if v.split() else ""
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return {}
    return vals


def bytes_per_ray(counts, hits):
    """Algorithmic bytes per ray of the hierarchical traversal, in the
    paper's node format (Section 3.2) and material scheme (Section 3.3), from
    the oracle's visit counts: 8 B (header word and child pointer) per
    internal node descended, the chunk's root included; 8 B per 4^3 leaf
    bitmap; at a hit, 4 B per preceding-sibling subtree count that the DFS
    index adds up, 4 B per run start the block search compares and 1 B of
    material; and the 16 B record."""
    b = (8.0 * (counts["chunk_entries"] + counts["node_cubes"]) + 8.0 * counts["leaf_cubes"] + 16.0)
    h = hits["hit"] == 1
    b[h] += 4.0 * counts["preceding_siblings"][h] + 4.0 * counts["run_probes"][h] + 1.0
    return b


def layout_bytes_per_ray(counts, hits, chunk_log2, sector=0):
    """Bytes per ray that this library's device layout reads for the same
    visits: 4 B view entry per chunk visited; 20 B per chunk DAG entered
    (node and leaf array addresses, root word); 4 B child word per internal
    node entered (the child's mask rides in its parent's word); 12 B (child
    word + bitmap) per leaf entered; at a hit 28 B (prefix and run array
    addresses, run count), one 4-B DFS prefix per internal level (the
    siblings' counts are summed ahead of time), 4 B per run start compared
    and 1 B material; the 16 B record.  With `sector` > 0 every one of those
    reads costs a whole sector of that many bytes instead (the no-reuse
    upper bound; the record stays 16 B)."""
    def rd(nbytes, accesses):
        return sector * accesses if sector else nbytes
    b = (rd(4.0, 1) * counts["chunk_visits"] + rd(20.0, 1) * counts["chunk_entries"] +
         rd(4.0, 1) * counts["node_cubes"] + rd(12.0, 2) * counts["leaf_cubes"] + 16.0)
    h = hits["hit"] == 1
    k = hits["lod"][h]
    b[h] += (rd(28.0, 1) + rd(4.0, 1) * (chunk_log2 - k - 2) + rd(4.0, 1) * counts["run_probes"][h] +
             rd(1.0, 1))
    return b


def host_cores():
    """(cores, nproc, cgroup limit): the CPUs this process may run on (what
    nproc reports), cut to the cgroup's CPU quota when one is set (threads
    beyond it would only time-slice)."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    limit = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            limit = int(q) / int(per)
    except (OSError, ValueError):
        pass
    cores = nproc if limit is None else max(1, min(nproc, int(limit)))
    return cores, nproc, limit


def build_chunks(args, sw, lod_count, gen, svdag, torch, ow=None, need=None):
    """Every chunk of the scene generated once (on the host, or on the GPU and
    copied into pinned host buffers) and built into a library blob (all
    LODs) by a pool of host threads; with an oracle world `ow`, the oracle's
    own DAGs of the LODs need[ci] are built from the same bytes and set in
    it (test infrastructure, for the CPU-baseline leg only)."""
    CL = sw.chunk_log2
    gx, gy, gz = sw.grid
    nch = gx * gy * gz
    t0 = time.time()
    blobs = {}
    if ow is not None:
        import oracle

    def work(ci, g=None):
        c = (ci % gx, (ci // gx) % gy, ci // (gx * gy))
        if g is None:
            g = sw.chunk(c, threads=1 if nch > 1 else args.threads)
        b = svdag.svd_chunk_build(g, CL, lod_count)
        odags = []
        if ow is not None and need[ci]:
            pyr = oracle.pyramid(g, 1 << CL, max(need[ci]) + 1)
            for k in sorted(need[ci]):
                odags.append((k, oracle.Dag(pyr[k], (1 << CL) >> k)))
        return ci, b, odags

    def gpu_generated(ex):
        """Chunks generated on the GPU one at a time (one S^3 device buffer),
        copied to a pinned host buffer and built by the pool; host buffers
        are recycled as builds finish."""
        import collections
        import queue
        S = 1 << CL
        dev = torch.empty(S ** 3, dtype=torch.uint8, device="cuda")
        free = queue.Queue()
        for _ in range(args.threads + 2):
            free.put(torch.empty(S ** 3, dtype=torch.uint8, pin_memory=True))
        work_dev = None

        def build_and_recycle(ci, h):
            try:
                return work(ci, h.numpy())
            finally:
                free.put(h)

        futs = collections.deque()
        for ci in range(nch):
            h = free.get()
            work_dev = sw.chunk_device((ci % gx, (ci // gx) % gy, ci // (gx * gy)), dev, work_dev)
            h.copy_(dev)  # synchronous: the buffer is complete when the build starts
            futs.append(ex.submit(build_and_recycle, ci, h))
            while futs and futs[0].done():
                yield futs.popleft().result()
        while futs:
            yield futs.popleft().result()

    with ThreadPoolExecutor(args.threads) as ex:
        results = gpu_generated(ex) if gen == "gpu" else ex.map(work, range(nch))
        for n_done, (ci, b, odags) in enumerate(results, 1):
            blobs[ci] = b
            for k, d in odags:
                ow.set_dag(ci, k, d)
            if n_done % 64 == 0:
                log(f"  {n_done}/{nch} chunks built ({time.time() - t0:.1f}s)")
    log(f"built {nch} chunks ({lod_count} LODs) in {time.time() - t0:.1f}s")
    return blobs


def make_world(sw, blobs, lod_count, thr, svdag, torch):
    """A world over a pool that holds every chunk LOD, all uploaded."""
    gx, gy, gz = sw.grid
    nch = gx * gy * gz
    desc = svdag.make_desc(sw.chunk_log2, sw.grid, lod_count, thr)
    dev_bytes = sum(svdag.svd_blob_stats_get(b, k)["device_bytes"] for b in blobs.values()
                    for k in range(lod_count))
    pool = torch.empty(svdag.table_bytes(sw.grid) + dev_bytes + 256 * nch * lod_count + (8 << 20),
                       dtype=torch.uint8, device="cuda")
    world = svdag.svd_world_create(desc, pool)
    for ci, b in blobs.items():
        svdag.svd_chunk_upload(world, (ci % gx, (ci // gx) % gy, ci // (gx * gy)), b)
    torch.cuda.synchronize()
    return world, pool, dev_bytes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="map512", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=2025)
    ap.add_argument("--views", type=int, default=10)
    ap.add_argument("--beam", action="store_true", help="trace with the beam pass (same records)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle legs (CPU baseline and visit counts)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU-baseline time")
    ap.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads that build the chunks")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the CPU baseline (0 = every core this process may use)")
    ap.add_argument("--batch-views", type=int, default=64,
                    help="views in the batched-launch comparison (0 = skip it)")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="length of each fixed-rate serving run (0 = skip the served comparison)")
    ap.add_argument("--serve-rates", default="2000", help="request arrival rates on the workload's map (req/s)")
    ap.add_argument("--serve-backlog", type=int, default=1000,
                    help="requests of the saturated run (as many in flight as output buffers)")
    ap.add_argument("--serve-pool-frac", type=float, default=0.25,
                    help="server pool for chunk data, as a fraction of the map's device bytes")
    ap.add_argument("--serve-views", type=int, default=64, help="requests per batched launch")
    ap.add_argument("--serve-inflight", type=int, default=2, help="launches in flight")
    ap.add_argument("--serve-max-rays", type=int, default=8 << 20, help="rays per batched launch")
    ap.add_argument("--serve-streaming-factor", type=float, default=1.5,
                    help="streaming factor of the prefetching runs (0 = skip them)")
    ap.add_argument("--serve-speed", type=float, default=600.0,
                    help="walker speed, voxels/s (fast enough that the walkers' chunk sets outgrow the pool)")
    ap.add_argument("--gen", choices=("host", "gpu"), default="host",
                    help="generate the scene's chunks on the host or with the GPU copy of the generator "
                         "(same bytes; gpu makes map1024 practical)")
    ap.add_argument("--other-workloads", default="terrain1024,noise64",
                    help="comma-separated workloads whose per-view leg also runs, without the oracle "
                         "legs ('' = none)")
    ap.add_argument("--c4-seconds", type=float, default=32.0,
                    help="length of each served run on map1024 (0 = skip that leg)")
    ap.add_argument("--c4-rate", type=float, default=200.0, help="request arrival rate on map1024 (req/s)")
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds the whole run may take: the map1024 leg is skipped (and said so) "
                         "if it would not fit")
    ap.add_argument("--tune-cache", default=default_tune_cache(),
                    help="tuning cache file of the per-view and batch tuners ('none': tune every run)")
    ap.add_argument("--view-tile", type=int, default=0, choices=(0, 8, 16, 32, 64),
                    help="per-view tile width (with --view-occupancy: no tuning; 0 = tuned)")
    ap.add_argument("--view-occupancy", type=int, default=0, help="per-view trace blocks per CU (0 = tuned)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    t_begin = time.time()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}))
        return
    for name in (w for w in args.other_workloads.split(",") if w):
        if name not in WORKLOADS:
            ap.error(f"--other-workloads: unknown workload {name!r}")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path does not "
              "shard across GPUs here (views would be routed to GPUs by chunk locality; there is no "
              "multi-GPU code).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2505_02017_amd import scenes, svdag
    svdag.lib()  # fails loudly if the HIP library is missing
    assert torch.cuda.is_available(), "no GPU"

    kind, lod_count, thr, wdesc = WORKLOADS[args.workload]
    sw = scenes.SceneWorld(kind, args.seed)
    CL = sw.chunk_log2
    gx, gy, gz = sw.grid
    nch = gx * gy * gz
    cams = sw.views(args.views, 1)
    W, H = cams[0].width, cams[0].height
    # The oracle (test infrastructure) runs only in this CPU-baseline leg:
    # its own DAGs of the sampled views, its timing on the host cores, its
    # visit counts (the algorithmic bytes of the roofline) and a spot check
    # of view 0.  Nothing it computes reaches the GPU path.
    use_oracle = not args.no_cpu_baseline

    # ---- oracle side: which (chunk, LOD) DAGs the sampled views need
    ow = None
    need = None
    if use_oracle:
        import oracle
        ow = oracle.World(CL, sw.grid, lod_count)
        frames = [oracle.camera_frame(c) for c in cams]
        view_lods = [ow.lod_pick(f.O, thr) for f in frames]
        need = [set() for _ in range(nch)]
        for vl in view_lods:
            for ci in range(nch):
                need[ci].add(int(vl[ci]))

    blobs = build_chunks(args, sw, lod_count, args.gen, svdag, torch, ow, need)
    world, pool, dev_bytes = make_world(sw, blobs, lod_count, thr, svdag, torch)
    log(f"uploaded {dev_bytes / 2**20:.1f} MiB of chunk DAGs")

    frames_gpu = [svdag.svd_camera_frame(c) for c in cams]
    out = torch.empty((W * H, 4), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    stage_flags = svdag.SVD_BEAM if args.beam else 0
    # the per-view tile and occupancy: from the tuning cache, else tuned on
    # the benchmark's own views (and stored), before the warm-up
    cache = tune_cache_path(args)
    if args.view_tile and args.view_occupancy:
        svdag.svd_world_set_tiling(world, args.view_tile)
        svdag.svd_world_set_occupancy(world, args.view_occupancy)
        view_tuning = {"tile": f"{args.view_tile}x{64 // args.view_tile}", "blocks_per_cu": args.view_occupancy,
                       "from_cache": False, "fixed": True}
        log(f"per-view tile {args.view_tile}x{64 // args.view_tile}, {args.view_occupancy} blocks/CU (fixed)")
    else:
        tuned, cache = tune_world(svdag, world, frames_gpu, out, stage_flags, cache, stream)
        view_tuning = tuned.as_dict()
        log(f"per-view tile {tuned.tile_w}x{64 // tuned.tile_w}, {tuned.blocks_per_cu} blocks/CU "
            + ("(from the tuning cache)" if tuned.from_cache else f"(tuned: {tuned.configs_timed} configurations)"))

    def step(i, ev=None):
        f = frames_gpu[i % len(frames_gpu)]
        if ev is not None:
            ev[0].record(stream)
        svdag.svd_view_stage(world, f, stage_flags, stream)
        if ev is not None:
            ev[1].record(stream)
        svdag.svd_view_beam(world, f, out, stream)
        if ev is not None:
            ev[2].record(stream)
        svdag.svd_view_trace(world, f, out, stream)
        if ev is not None:
            ev[3].record(stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    # Timed region.  Each step's trace pass (beam kernel, if any, + trace
    # kernel) is timed by HIP events that the library stamps from the
    # kernels' own dispatches on this stream (svd_world_time_traces): event
    # markers between the launches would each add idle time to the steps.
    svdag.svd_world_time_traces(world, args.steps)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    pass_ms = np.array(svdag.svd_world_trace_times(world, args.steps), dtype=np.float64)
    svdag.svd_world_time_traces(world, 0)
    assert pass_ms.size == args.steps, "trace passes not all timed"
    rays = W * H * args.steps
    value = rays / t_total / 1e9
    # Per-kernel and per-view times, outside the timed region: the same steps
    # again with event markers around each kernel.
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for i in range(args.steps):
        step(i, evs[i])
    torch.cuda.synchronize()
    stage_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    beam_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    trace_ms = np.array([e[2].elapsed_time(e[3]) for e in evs])
    view_ms = stage_ms + beam_ms + trace_ms
    if not args.beam:
        trace_ms = pass_ms  # the trace kernel alone, as timed in the timed region

    # beside the metric: views whose records are also copied to pinned host
    # memory (stage + trace + D2H on the same stream), outside the timed region
    host = torch.empty((W * H, 4), dtype=torch.int32, pin_memory=True)
    nd2h = min(args.steps, 10)
    evd = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(nd2h)]
    for i in range(nd2h):
        evd[i][0].record(stream)
        step(i)
        host.copy_(out, non_blocking=True)
        evd[i][1].record(stream)
    torch.cuda.synchronize()
    d2h_ms = np.array([e[0].elapsed_time(e[1]) for e in evd])

    raw = out.cpu().numpy()
    hits = svdag.decode_hits(raw)
    assert not np.any(hits["chunk"] == svdag.FAULT_CHUNK), "iteration guard fired"

    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Grays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_total * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wdesc, "chunks": nch, "chunk_edge": 1 << CL, "lods": lod_count,
                   "width": W, "height": H, "views": len(cams), "seed": args.seed,
                   "chunks_generated_on": args.gen},
        "p50_view_ms": round(float(np.percentile(view_ms, 50)), 4),
        "p99_view_ms": round(float(np.percentile(view_ms, 99)), 4),
        "trace_kernel_ms_mean": round(float(trace_ms.mean()), 4),
        "beam_kernel_ms_mean": round(float(beam_ms.mean()), 4),
        "stage_kernel_ms_mean": round(float(stage_ms.mean()), 4),
        "beam_pass": bool(args.beam),
        "with_d2h": {"p50_view_ms": round(float(np.percentile(d2h_ms, 50)), 4),
                     "grays": round(W * H / float(np.percentile(d2h_ms, 50)) / 1e6, 4),
                     "note": "stage + trace + records to pinned host memory (PCIe), not the metric"},
        "hit_fraction": round(float(hits["hit"].mean()), 4),
        "tuning": {"kernel_hash": svdag.svd_kernel_hash(), "cache": cache, "view": view_tuning},
    }

    if use_oracle:
        cores, nproc, cg_limit = host_cores()
        cpu_threads = args.cpu_threads or cores
        # ---- algorithmic bytes per ray: oracle visit counts on a sparse sample of every view
        stride = 97
        per_ray, per_ray_layout, per_ray_sec = [], [], []
        for v, f in enumerate(frames):
            idx = np.arange(v % stride, W * H, stride, dtype=np.uint32)
            h, cnt = ow.trace_frame(view_lods[v], f, idx, mode=1, threads=cpu_threads, counts=True)
            per_ray.append(bytes_per_ray(cnt, h))
            per_ray_layout.append(layout_bytes_per_ray(cnt, h, CL))
            per_ray_sec.append(layout_bytes_per_ray(cnt, h, CL, sector=64))
        # per-view launches cycle over the views; weight each view's bytes by its launches
        nviews = len(frames)
        launches = np.bincount(np.arange(args.steps) % nviews, minlength=nviews)

        def per_launch(rays_bytes):
            view_b = np.array([p.mean() for p in rays_bytes])
            return float((view_b * launches).sum() / launches.sum()) * W * H
        bytes_per_launch = per_launch(per_ray)
        layout_per_launch = per_launch(per_ray_layout)
        # compulsory bytes: every part of the device layout a view's rays
        # touch, counted once (child words, leaf bitmaps, prefix counts, run
        # starts and materials, view-table entries, 64-B descriptors), plus
        # the records
        comp = []
        for v, f in enumerate(frames):
            t = ow.touch_frame(view_lods[v], f, threads=cpu_threads)
            comp.append(4 * t["child_words"] + 8 * t["leaves"] + 4 * t["prefixes"] + 4 * t["run_starts"] +
                        t["run_materials"] + 4 * t["chunks"] + 64 * t["dags"] + 16 * t["rays"])
        compulsory = float((np.array(comp, np.float64) * launches).sum() / launches.sum())
        launch_s = pass_ms.mean() * 1e-3
        achieved = bytes_per_launch / launch_s / 1e9
        prof = counter_profile(args.workload)
        traffic = float(prof["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in prof else None
        result["roofline"] = {
            "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": round(traffic) if traffic is not None else None,
            "kernel": "beam_kernel + trace_kernel" if args.beam else "trace_kernel",
            "launch_ms": round(float(pass_ms.mean()), 4),
            # frac: the paper's node format and DFS resolve (preceding-sibling
            # counts), from the oracle's pinned visit counts
            "bytes_per_ray": round(float(np.concatenate(per_ray).mean()), 2),
            "bytes_per_launch": round(bytes_per_launch),
            # the same visits in this library's device layout
            "layout_bytes_per_ray": round(float(np.concatenate(per_ray_layout).mean()), 2),
            "layout_frac": round(layout_per_launch / launch_s / 1e9 / HBM_PEAK_GBS, 5),
            # no-reuse upper bound: every layout read a whole 64-B sector
            "sector64_bytes_per_ray": round(float(np.concatenate(per_ray_sec).mean()), 2),
            # compulsory lower bound: each touched byte once (records included)
            "compulsory_bytes_per_launch": round(compulsory),
            "record_bytes_per_launch": W * H * 16,
            # what HBM actually moved (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)
            "hbm_measured_gbs": round(traffic / launch_s / 1e9, 2) if traffic is not None else None,
            "hbm_measured_frac": round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 5) if traffic is not None else None,
            "blocks_per_cu": int(svdag.svd_world_get_occupancy(world)[0]),
        }
        if "l1_hit_rate" in prof:
            result["caches"] = {"l1_hit_rate": float(prof["l1_hit_rate"]), "l2_hit_rate": float(prof["l2_hit_rate"]),
                                "source": "rocprofv3 TCP/TCC counters in profiles/ (same kernel source)"}
            if "mall_hit_rate" in prof:
                result["caches"]["mall_hit_rate"] = float(prof["mall_hit_rate"])
        if "valu_insts_per_launch" in prof:
            # VALU issue view: wave instructions per second over the issue peak
            # (1024 SIMDs x 2.4 GHz / 4 cycles per wave64 VALU instruction)
            rate = float(prof["valu_insts_per_launch"]) / (trace_ms.mean() * 1e-3)  # trace kernel alone
            peak = 1024 * 2.4e9 / 4
            result["valu_issue"] = {"achieved": round(rate / 1e9, 2), "peak": round(peak / 1e9, 2),
                                    "unit": "G wave-instructions/s", "frac": round(rate / peak, 4),
                                    "insts_per_launch": int(float(prof["valu_insts_per_launch"]))}
            if "valu_lane_utilisation" in prof:
                result["valu_issue"]["lane_utilisation"] = float(prof["valu_lane_utilisation"])
            if "shader_clock_ghz" in prof:
                # the same issue rate against the clock the chip ran the
                # kernel at, and the share of the launch its CUs were busy
                # (SQ / GRBM cycle counters of the same kernel source)
                clk = float(prof["shader_clock_ghz"])
                result["valu_issue"]["shader_clock_ghz"] = clk
                result["valu_issue"]["frac_at_measured_clock"] = round(rate / (1024 * clk * 1e9 / 4), 4)
                if "cu_busy_fraction" in prof:
                    result["valu_issue"]["cu_busy_fraction"] = float(prof["cu_busy_fraction"])
            # the unit that binds: VALU issue, not HBM
            result["roofline"]["limiter"] = {"unit": "valu_issue", "frac": round(rate / peak, 4)}
        # ---- CPU baseline: the oracle (as is) on a bounded sample: whole views
        #      in benchmark order while the time budget lasts (repeated passes
        #      over all of them if they fit more than once, at most 8), else
        #      evenly spaced pixels of view 0
        pilot = np.arange(0, W * H, max(1, (W * H) // 4000), dtype=np.uint32)
        t = time.perf_counter()
        ow.trace_frame(view_lods[0], frames[0], pilot, mode=1, threads=cpu_threads)
        per = (time.perf_counter() - t) / pilot.size
        n_budget = int(max(1000, args.cpu_seconds / max(per, 1e-12)))
        nviews_cpu = max(1, min(nviews, n_budget // (W * H)))
        n0 = W * H if n_budget >= W * H else n_budget
        sample0 = np.linspace(0, W * H - 1, n0).astype(np.uint32)
        t = time.perf_counter()
        passes = 0
        while True:
            refs = [ow.trace_frame(view_lods[v], frames[v], sample0 if v == 0 else None, mode=1,
                                   threads=cpu_threads) for v in range(nviews_cpu)]
            passes += 1
            dt = time.perf_counter() - t
            # another pass over all views only if it still fits the budget
            if nviews_cpu < nviews or passes >= 8 or dt * (passes + 1) / passes > args.cpu_seconds:
                break
        n = passes * (n0 + (nviews_cpu - 1) * W * H)
        # view 0 of the sample doubles as a parity spot-check of the benchmarked path
        step(0)
        torch.cuda.synchronize()
        g = svdag.decode_hits(out.cpu().numpy())
        ref = refs[0]
        result["cpu_sample_parity"] = bool(all(
            np.array_equal(np.where(ref["hit"] == 1, ref[f], 0), g[f][sample0])
            for f in ("hit", "x", "y", "z", "lod", "face", "material")))
        what = (f"all pixels of views 0..{nviews_cpu - 1}" if n0 == W * H
                else f"{n0} evenly spaced pixels of view 0")
        if passes > 1:
            what += f", {passes} passes"
        result["cpu_baseline"] = {
            "value": round(n / dt / 1e9, 6), "unit": "Grays/s", "cores": cpu_threads,
            "kind": "oracle",
            "sample": f"{n} rays: {what} ({W}x{H}), oracle mode 1 (empty-subtree skipping), "
                      f"{cpu_threads} threads, {dt:.1f}s",
            "nproc": nproc, "cgroup_cpu_limit": cg_limit,
        }

    if args.batch_views > 0:
        result["batched"] = bench_batched(args, sw, world, svdag, torch, cache)
        result["tuning"]["batch"] = result["batched"].pop("tuning")
    modes = ("batched", "plain", "plain_concurrent")
    if args.serve_seconds > 0:
        # the workload's own map: rates where the walkers outgrow the pool
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        result["served"] = bench_served(args, sw, blobs, lod_count, thr, world, svdag, torch, rates,
                                        args.serve_seconds, modes, args.serve_backlog,
                                        args.serve_streaming_factor)
    del world, pool, out
    blobs.clear()
    ow = None
    torch.cuda.empty_cache()
    others = [w for w in args.other_workloads.split(",") if w and w != args.workload]
    if others:
        result["other_workloads"] = {}
        for name in others:
            result["other_workloads"][name] = bench_other_workload(args, name, svdag, torch, cache)
            torch.cuda.empty_cache()
    if args.c4_seconds > 0 and args.workload != "map1024":
        # the served configuration: 32x32 chunks of 1024^3, pool at a quarter
        # of the map, Poisson arrivals at 200 requests/s from walkers
        elapsed = time.time() - t_begin
        need_s = 150 + 4 * args.c4_seconds
        if elapsed + need_s > args.time_budget:
            result["served_map1024"] = {"skipped": f"time budget: {elapsed:.0f} s spent, about {need_s:.0f} s "
                                                   f"more needed, {args.time_budget:.0f} s allowed"}
        else:
            kind4, lods4, thr4, desc4 = WORKLOADS["map1024"]
            sw4 = scenes.SceneWorld(kind4, args.seed)
            blobs4 = build_chunks(args, sw4, lods4, "gpu", svdag, torch)
            world4, pool4, bytes4 = make_world(sw4, blobs4, lods4, thr4, svdag, torch)
            log(f"map1024: uploaded {bytes4 / 2**30:.2f} GiB of chunk DAGs")
            r = bench_served(args, sw4, blobs4, lods4, thr4, world4, svdag, torch, [args.c4_rate],
                             args.c4_seconds, modes, args.serve_backlog, args.serve_streaming_factor)
            r["workload"] = desc4.split(", 2560x1440")[0] + ", chunks generated on the GPU"
            result["served_map1024"] = r
            del world4, pool4
            blobs4.clear()
            torch.cuda.empty_cache()
    result["bench_seconds"] = round(time.time() - t_begin, 1)

    print(json.dumps(result), flush=True)


def bench_other_workload(args, name, svdag, torch, cache):
    """The per-view leg alone on another workload (chunks generated on the
    host, every LOD resident; tile and occupancy tuned or from the cache):
    the same timed steps as the headline, without the oracle legs."""
    from paper_2505_02017_amd import scenes
    t0 = time.time()
    kind, lod_count, thr, wdesc = WORKLOADS[name]
    sw = scenes.SceneWorld(kind, args.seed)
    cams = sw.views(args.views, 1)
    W, H = cams[0].width, cams[0].height
    blobs = build_chunks(args, sw, lod_count, "host", svdag, torch)
    world, pool, _ = make_world(sw, blobs, lod_count, thr, svdag, torch)
    frames = [svdag.svd_camera_frame(c) for c in cams]
    out = torch.empty((W * H, 4), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    tuned, _ = tune_world(svdag, world, frames, out, 0, cache, stream)

    def step(i):
        f = frames[i % len(frames)]
        svdag.svd_view_stage(world, f, 0, stream)
        svdag.svd_view_trace(world, f, out, stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    svdag.svd_world_time_traces(world, args.steps)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    trace_ms = np.array(svdag.svd_world_trace_times(world, args.steps), dtype=np.float64)
    svdag.svd_world_time_traces(world, 0)
    hits = svdag.decode_hits(out.cpu().numpy())
    assert not np.any(hits["chunk"] == svdag.FAULT_CHUNK), "iteration guard fired"
    r = {"workload": wdesc, "value": round(W * H * args.steps / dt / 1e9, 4), "unit": "Grays/s",
         "steps": args.steps, "ms_per_step": round(dt * 1e3 / args.steps, 4),
         "trace_kernel_ms_mean": round(float(trace_ms.mean()), 4),
         "tile": f"{tuned.tile_w}x{64 // tuned.tile_w}", "blocks_per_cu": tuned.blocks_per_cu,
         "tuning_from_cache": bool(tuned.from_cache), "hit_fraction": round(float(hits["hit"].mean()), 4),
         "seconds": round(time.time() - t0, 1)}
    log(f"{name}: {r['value']} Grays/s, trace {r['trace_kernel_ms_mean']} ms, tile {r['tile']}, "
        f"{r['blocks_per_cu']} blocks/CU")
    del world, pool
    return r


def bench_batched(args, sw, world, svdag, torch, cache):
    """A batch of views of mixed resolution over the same world: one
    graph-launched batch (autotuned tiling) against per-view launches."""
    rng = np.random.default_rng([args.seed, 64])
    sizes = [(320, 180), (640, 360), (1280, 720), (1920, 1080)]
    cams = []
    for i in range(args.batch_views):
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        cams.append(sw.views(1, 1000 + i, W, H)[0])
    nrec = svdag.batch_records(cams)
    frames = [svdag.svd_camera_frame(c) for c in cams]
    offs = np.concatenate([[0], np.cumsum([c.width * c.height for c in cams])])
    out_b = torch.empty((nrec, 4), dtype=torch.int32, device="cuda")
    out_p = torch.empty((nrec, 4), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    batch = svdag.svd_batch_create(world, len(cams))
    try:
        tuned = svdag.svd_batch_tune_cached(batch, cams, out_b, reps=3, cache_path=cache, stream=stream)
    except svdag.SvdError as e:
        if e.code != svdag.SVD_EIO:
            raise
        log(f"tuning cache not written ({e}); tuning without it")
        tuned = svdag.svd_batch_tune_cached(batch, cams, out_b, reps=3, cache_path=None, stream=stream)
    tw, claim, occ = tuned.tile_w, tuned.claim, tuned.blocks_per_cu
    log(f"batch of {len(cams)} views ({nrec} rays): tile {tw}x{64 // tw}, claim {claim}, {occ} blocks/CU "
        + ("(from the tuning cache)" if tuned.from_cache else f"(tuned: {tuned.configs_timed} configurations)"))

    def plain():
        for v, f in enumerate(frames):
            svdag.svd_trace_frame(world, f, out_p[offs[v]:offs[v + 1]], 0, stream)

    def batched():
        svdag.svd_batch_trace_frames(batch, frames, out_b, 0, stream)

    res = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.batch_reps)]
        t0 = time.perf_counter()
        for e in ev:
            e[0].record(stream)
            fn()
            e[1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
        res[name] = (wall, ms)
    identical = bool(torch.equal(out_b, out_p))
    svdag.svd_batch_destroy(batch)
    wb, mb = res["batched"]
    wp, mp = res["plain"]
    return {
        "views": len(cams), "rays_per_batch": int(nrec), "resolutions": "uniform over 320x180, 640x360, "
        "1280x720, 1920x1080", "tile": f"{tw}x{64 // tw}", "claim": claim,
        "blocks_per_cu": occ,
        "batched_grays": round(nrec * args.batch_reps / wb / 1e9, 4),
        "plain_grays": round(nrec * args.batch_reps / wp / 1e9, 4),
        "speedup": round(wp / wb, 3),
        "batched_ms_p50": round(float(np.percentile(mb, 50)), 4),
        "batched_ms_p99": round(float(np.percentile(mb, 99)), 4),
        "plain_ms_p50": round(float(np.percentile(mp, 50)), 4),
        "plain_ms_p99": round(float(np.percentile(mp, 99)), 4),
        "identical_to_plain": identical,
        "tuning": tuned.as_dict(),
    }


def bench_served(args, sw, blobs, lod_count, thr, full_world, svdag, torch, rates, seconds, modes, backlog,
                 prefetch_sf):
    """Served requests over a pool that holds a fraction of the map's chunk
    LODs: walkers issue Poisson-arriving views of mixed resolution; batched
    continuous serving against per-request plain launches (serial on one
    stream, and concurrent on the flights' own streams and tables) on the
    same schedule, at fixed rates and saturated (as many requests in flight
    as there are output buffers).  Latency = completion seen by the server's
    worker minus the request's scheduled arrival."""
    import threading
    gx, gy, gz = sw.grid
    nch = gx * gy * gz
    CL = sw.chunk_log2
    coords = [(ci % gx, (ci // gx) % gy, ci // (gx * gy)) for ci in range(nch)]
    all_bytes = sum((svdag.svd_blob_stats_get(b, k)["device_bytes"] + 255) // 256 * 256
                    for b in blobs.values() for k in range(lod_count))
    budget = int(args.serve_pool_frac * all_bytes) // 256 * 256
    ring, maxpx = 256, 1920 * 1080
    outs = torch.empty((ring, maxpx, 4), dtype=torch.int32, device="cuda")
    desc = svdag.make_desc(CL, sw.grid, lod_count, thr)
    views, inflight = args.serve_views, args.serve_inflight
    old_switch = sys.getswitchinterval()
    sys.setswitchinterval(0.0005)

    def run(mode, schedule, backlog, sf=0.0):
        pool = torch.empty(svdag.table_bytes(sw.grid) + inflight * svdag.batch_bytes(nch, views) + budget,
                           dtype=torch.uint8, device="cuda")
        w = svdag.svd_world_create(desc, pool)
        s = svdag.svd_server_create(w, mode=mode, max_views=views, inflight=inflight,
                                    max_rays=args.serve_max_rays, streaming_factor=sf)
        for ci, b in blobs.items():
            svdag.svd_server_set_chunk(s, coords[ci], b)
        torch.cuda.synchronize()
        n = len(schedule)
        late = np.zeros(n)
        busy = np.zeros(ring, bool)
        cv = threading.Condition()
        done = {}

        def submitter():
            t0 = time.perf_counter()
            for i, (t, cam) in enumerate(schedule):
                j = i % ring
                with cv:
                    while busy[j]:
                        cv.wait(0.01)
                    busy[j] = True
                if not backlog:
                    target = t0 + t
                    while True:
                        d = target - time.perf_counter()
                        if d <= 0:
                            break
                        if d > 0.001:
                            time.sleep(d - 0.0008)
                    late[i] = time.perf_counter() - target
                svdag.svd_server_submit(s, cam, outs[j], tag=i)

        th = threading.Thread(target=submitter)
        th.start()
        while len(done) < n:
            for d in svdag.svd_server_poll(s, 1024, wait_us=20000):
                done[d["tag"]] = d
                with cv:
                    busy[d["tag"] % ring] = False
                    cv.notify_all()
        th.join()
        st = svdag.svd_server_stats_get(s)
        svdag.svd_server_destroy(s)
        torch.cuda.synchronize()
        failed = sum(1 for d in done.values() if d["status"] != 0)
        lat = np.array([done[i]["t_done"] - done[i]["t_submit"] + late[i] for i in range(n)]) * 1e3
        warm = np.array([t >= 1.0 for t, _ in schedule]) if not backlog else np.ones(n, bool)
        rays = sum(c.width * c.height for _, c in schedule)
        span = max(d["t_done"] for d in done.values()) - min(d["t_submit"] for d in done.values())
        bv = np.array([d["batch_views"] for d in done.values()])
        r = {"requests": n, "failed": failed, "grays": round(rays / span / 1e9, 4),
             "p50_ms": round(float(np.percentile(lat[warm], 50)), 3),
             "p99_ms": round(float(np.percentile(lat[warm], 99)), 3),
             "measured_requests": int(warm.sum()),
             "mean_requests_per_launch": round(float(bv.mean()), 2), "launches": st["launches"],
             "uploads": st["uploads"], "upload_mib": round(st["upload_bytes"] / 2**20, 1),
             "evictions": st["evictions"], "memory_waits": st["memory_waits"],
             "prefetches": st["prefetches"], "prefetch_mib": round(st["prefetch_bytes"] / 2**20, 1)}
        # the last requests' records are still in the output ring: each equals its view traced alone
        ok = True
        for i in range(max(0, n - 8), n):
            cam = schedule[i][1]
            alone = torch.empty((cam.width * cam.height, 4), dtype=torch.int32, device="cuda")
            svdag.svd_trace_view(full_world, svdag.to_camera(cam), alone)
            torch.cuda.synchronize()
            ok &= bool(torch.equal(alone, outs[i % ring, :cam.width * cam.height]))
        r["last8_identical_to_alone"] = ok
        return r

    res = {"pool_bytes_for_chunks": budget, "map_bytes_all_lods": all_bytes,
           "pool_fraction": args.serve_pool_frac, "walkers": 8, "walker_speed": args.serve_speed,
           "seconds_per_run": seconds,
           "resolutions": "uniform over 320x180, 640x360, 1280x720, 1920x1080",
           "batched_launch": {"max_requests": views, "max_rays": args.serve_max_rays, "inflight": inflight},
           "plain": "one stage + trace pair per request, serial on one stream",
           "plain_concurrent": f"one stage + trace pair per request, up to {inflight} at once on their own "
                               "streams and view tables",
           "prefetch_streaming_factor": prefetch_sf,
           "latency": "scheduled arrival to completion; requests arriving in the first second "
                      "(cold pool) are served but not in the percentiles"}
    mode_ids = {"batched": svdag.SVD_SERVE_BATCHED, "plain": svdag.SVD_SERVE_PLAIN,
                "plain_concurrent": svdag.SVD_SERVE_PLAIN_CONCURRENT}
    for rate in rates:
        sched = sw.walk_requests(8, rate, seconds, seed=int(rate), speed=args.serve_speed)
        for name in modes:
            log(f"serving {len(sched)} requests at {rate:g}/s, {name}")
            res[f"{name}_{rate:g}rps"] = run(mode_ids[name], sched, False)
        if prefetch_sf > 0:
            log(f"serving {len(sched)} requests at {rate:g}/s, batched with prefetch")
            res[f"batched_prefetch_{rate:g}rps"] = run(svdag.SVD_SERVE_BATCHED, sched, False, prefetch_sf)
    sched = sw.walk_requests(8, 400.0, backlog / 400.0 + 1.0, seed=99, speed=args.serve_speed)[:backlog]
    for name in (modes if backlog > 0 else ()):
        log(f"serving {len(sched)} requests saturated, {name}")
        res[f"{name}_saturated"] = run(mode_ids[name], sched, True)
    sys.setswitchinterval(old_switch)
    del outs
    return res


if __name__ == "__main__":
    main()
