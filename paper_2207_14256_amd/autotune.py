"""Autotuner for the push launch shape and the particle re-sort policy.

Candidates are timed on the device through the C ABI's own HIP-event timers:

  1. launch shape -- particles per thread and the cap on resident waves per
     SIMD, then the particles per thread of the push fused with a re-sort --
     over the full schedule, scored by the time of both push kernels;
  2. sort policy -- bucket size and the drift threshold of the adaptive
     cadence -- over the full schedule, since the cost of a stale order and the
     number of re-sorts both depend on how far the particles travel;
  3. a persistent push grid (a fixed number of blocks looping over the
     chunks) against one block per chunk, then hipGraph capture and replay of
     the step sequence against plain launches, both by wall time over the
     schedule.

Results are cached in ``tuning_cache.json`` next to this file, keyed by the
device architecture, mesh size, particles per cell, precision and number of
species.  None of the parameters changes results (the push is per particle
and the sort only permutes), only speed.
"""
import json
import os
import time

from . import fastdf

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def cache_key(cfg):
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    n = sum(int(sp["n_side"]) ** 3 for sp in cfg["species"])
    return "%s|G=%d|N/G3=%.4g|%s|species=%d|steps=%d" % (
        arch, cfg["grid_n"], n / cfg["grid_n"] ** 3, cfg["precision"], len(cfg["species"]), cfg["n_steps"])


def load_cache(path=CACHE_PATH):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def cached_tuning(cfg, path=CACHE_PATH):
    return load_cache(path).get(cache_key(cfg))


def _run(ctx, cfg, tuning, steps):
    import torch
    fastdf.setup_workload(cfg, ctx=ctx)
    ctx.set_tuning(**tuning)
    ctx.timing(not tuning.get("use_graph"))
    ctx.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    push_ms, launches = ctx.read_timing("push")
    ps_ms, _ = ctx.read_timing("push_sort")
    sort_ms, sorts = ctx.read_timing("sort")
    return dict(wall_s=wall, push_ms=push_ms / max(launches, 1), push_total_ms=push_ms + ps_ms,
                sort_ms=sort_ms, sorts=sorts)


def autotune(cfg, path=CACHE_PATH, log=print, full_schedule=True):
    """Time the candidates for this workload, store the best in the cache and
    return it (a dict accepted by Context.set_tuning)."""
    ctx = fastdf.Context(cfg)
    sorting = cfg.get("sort_every", 0) > 0
    base = dict(particles_per_thread=4, sort_tiles=0, sort_every=cfg.get("sort_every", 0),
                sort_cells=3.0 if sorting else 0.0, persistent_blocks=0, use_graph=0, sort_predict=1,
                sort_fused=1, push_waves=0, sort_push_ppt=1, sort_keys_push=1)
    # 1. launch shape: particles per thread and the cap on resident waves,
    #    timed over the whole schedule (the mesh locality of the gathers, and
    #    with it the best shape, changes as the particles disperse), scored
    #    by the time of both push kernels together.
    best, best_ms = None, float("inf")
    steps = cfg["n_steps"] if full_schedule else min(40, cfg["n_steps"])
    for ppt in (1, 2, 4, 8):
        for waves in (0, 2, 3, 4):
            t = dict(base, particles_per_thread=ppt, push_waves=waves)
            r = _run(ctx, cfg, t, steps)
            log("[autotune] ppt=%d push_waves=%d: push %.3f ms per launch, %.1f ms both push kernels" % (
                ppt, waves, r["push_ms"], r["push_total_ms"]))
            if r["push_total_ms"] < best_ms:
                best, best_ms = t, r["push_total_ms"]
    #    then the particles per thread of the fused re-sort push
    if sorting:
        for sppt in (2, 4):
            t = dict(best, sort_push_ppt=sppt)
            r = _run(ctx, cfg, t, steps)
            log("[autotune] sort_push_ppt=%d: %.1f ms both push kernels" % (sppt, r["push_total_ms"]))
            if r["push_total_ms"] < best_ms:
                best, best_ms = t, r["push_total_ms"]
    # 2. sort policy over the whole schedule
    if sorting and full_schedule:
        G = cfg["grid_n"]
        best_wall = float("inf")
        chosen = best
        for tiles in sorted({max(1, G // 8), max(1, G // 4), min(256, max(1, G // 2))}):
            for cells in (2.0, 3.0, 4.0, 6.0, 8.0, 16.0):
                t = dict(best, sort_tiles=min(tiles, 256), sort_cells=cells)
                r = _run(ctx, cfg, t, cfg["n_steps"])
                log("[autotune] tiles=%d cells=%.1f: %.3f s (push %.3f ms, %d sorts, %.0f ms sorting)" % (
                    tiles, cells, r["wall_s"], r["push_ms"], r["sorts"], r["sort_ms"]))
                if r["wall_s"] < best_wall:
                    chosen, best_wall = t, r["wall_s"]
        best = chosen
    # 3. a persistent push grid, then the launch sequence captured in a
    #    hipGraph and replayed, against plain launches, by wall time over the
    #    schedule (two runs each: the first replay of a graph includes its
    #    capture); either must win by 1 % (graphs turn the per-kernel timers
    #    off)
    if full_schedule:
        walls = {}
        for pb in (0, 1024, 2048):
            t = dict(best, persistent_blocks=pb)
            walls[pb] = min(_run(ctx, cfg, t, cfg["n_steps"])["wall_s"] for _ in range(2))
            log("[autotune] persistent_blocks=%d: %.3f s" % (pb, walls[pb]))
        pb = min(walls, key=walls.get)
        best = dict(best, persistent_blocks=pb if walls[pb] < 0.99 * walls[0] else 0)
        walls = {}
        for g in (0, 1):
            t = dict(best, use_graph=g)
            walls[g] = min(_run(ctx, cfg, t, cfg["n_steps"])["wall_s"] for _ in range(2))
            log("[autotune] use_graph=%d: %.3f s" % (g, walls[g]))
        best = dict(best, use_graph=int(walls[1] < 0.99 * walls[0]))
    ctx.close()
    cache = load_cache(path)
    cache[cache_key(cfg)] = best
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return best


def main(argv=None):
    import argparse
    import sys

    import torch

    from . import workloads
    ap = argparse.ArgumentParser(description="autotune a workload preset and store the result")
    ap.add_argument("workload")
    ap.add_argument("--cache", default=CACHE_PATH)
    ap.add_argument("--launch-only", action="store_true", help="short launch-shape runs, no sort sweep")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default=None,
                    help="override the preset's precision")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    cfg = workloads.preset(args.workload)
    if args.precision:
        cfg["precision"] = args.precision
    best = autotune(cfg, path=args.cache, full_schedule=not args.launch_only,
                    log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps({cache_key(cfg): best}))


if __name__ == "__main__":
    main()
