#!/usr/bin/env python3
"""Benchmark of the FastDF neutrino push on one MI355X.

One bench "step" is one whole job of the hot path on resident synthetic
input: seeded field, particle sample, potential grids (Fourier stage + 3-D
C2R FFT), the full leapfrog schedule (one push launch per step), delta-f
weights, and the CIC-deposit + binned cross power spectrum.  The default
workload is the precision form: 512^3 neutrinos (m = 0.1 eV) on a 512^3
bfloat16 gradient mesh in a 1 Gpc box, 1000 steps from z = 1e9 to z = 0,
FP32 push with 32-bit fixed-point positions and momenta kept as the initial
momentum plus the accumulated kicks.

Printed: one JSON line with particle-updates/s over the whole job, the push
kernel's achieved HBM bandwidth against the 8 TB/s peak (from HIP events on
the library's stream), the same job in the FP64 form for the speedup and the
P(k) difference, and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload c3] [--no-fp64-leg]
                    [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "particle-updates/s & HBM GB/s, FP32-fixed-pt vs FP64 push at stated P(k) error"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def mesh_slots(cfg):
    """(stored slots per cell, slots that carry data): grad psi (3), grad phi
    (3, when psi != phi) and phi-dot (1, when the potentials depend on time);
    cells with phi-dot = 0 keep 6 (bfloat16 ones 8 with pad_mesh)."""
    slip = bool(cfg.get("slip_amp", 0.0))
    tdep = cfg.get("model") == "radmat"
    data = 3 + (3 if slip else 0) + (1 if tdep else 0)
    if not slip:
        stored = 4
    elif (cfg["precision"] == "fp64" or not cfg.get("pad_mesh")) and not tdep:
        stored = 6
    else:
        stored = 8
    return stored, data


def state_bytes(cfg, drift):
    """Algorithmic state bytes of one particle-update: FP32 form read x, q0,
    dq (36 B), write x, dq (24 B; 12 B on a kick-only launch); FP64 form read
    x, q, q0 (72 B), write x, q (48 B; 24 B kick-only)."""
    if cfg["precision"] == "fp32":
        return 36 + (24 if drift else 12)
    return 72 + (48 if drift else 24)


def mesh_cell_bytes(cfg):
    """Algorithmic bytes of one mesh cell read: its slots that carry data (the
    zero phi-dot slot and the pad of a bfloat16 cell are traffic, not
    algorithm: see mesh_padding_bytes)."""
    _, data = mesh_slots(cfg)
    return data * (2 if cfg["precision"] == "fp32" else 8)


def bytes_per_launch(cfg, n_particles, drift):
    """Algorithmic HBM bytes of one push launch over n_particles of one
    field: state read + write per particle plus one read of the mesh."""
    return n_particles * state_bytes(cfg, drift) + cfg["grid_n"] ** 3 * mesh_cell_bytes(cfg)


def mesh_padding_bytes(cfg):
    """Bytes per mesh of slots read but carrying no data."""
    stored, data = mesh_slots(cfg)
    return cfg["grid_n"] ** 3 * (stored - data) * (2 if cfg["precision"] == "fp32" else 8)


SORT_PUSH_STATE_BYTES = 92   # x, q0, dq, id and the rank outputs read; the 40 B state written


def bytes_per_push_sort(cfg, n_particles):
    """Algorithmic HBM bytes of one push launch that also carries out a
    re-sort (FP32 form): the push's reads (x, q0, dq: 36 B), the id and the
    rank pass outputs (source slot, bucket, rank: 16 B) read, the whole state
    written in sorted order (40 B), and one read of the mesh's data slots."""
    return n_particles * SORT_PUSH_STATE_BYTES + cfg["grid_n"] ** 3 * mesh_cell_bytes(cfg)


def run_leg(cfg, steps, warmup, label, tuning=None):
    import torch
    from paper_2207_14256_amd import fastdf
    n_total = sum(int(sp["n_side"]) ** 3 for sp in cfg["species"])
    ctx = fastdf.Context(cfg)
    wbuf = torch.empty(max(int(sp["n_side"]) ** 3 for sp in cfg["species"]),
                       dtype=torch.float64, device="cuda")

    def job():
        _, fields, species = fastdf.setup_workload(cfg, ctx=ctx, tuning=tuning)
        ctx.step(cfg["n_steps"])
        for s in species:
            ctx.weights(s, out=wbuf)
        # one total spectrum per field (the species of one field share it);
        # the first field's is returned
        groups = {}
        for s, sp in zip(species, cfg["species"]):
            groups.setdefault(sp["field"], []).append(s)
        pks = [ctx.power_spectrum(g, cfg["pk_bins"], "cross") for _, g in sorted(groups.items())]
        return pks[0]

    for i in range(warmup):
        job()
        log("%s warmup %d/%d done" % (label, i + 1, warmup))
    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pk = None
    for i in range(steps):
        pk = job()
        log("%s step %d/%d done" % (label, i + 1, steps))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    push_ms, launches = ctx.read_timing("push")
    ps_ms, ps_launches = ctx.read_timing("push_sort")
    work_push, work_ps = ctx.read_work("push"), ctx.read_work("push_sort")
    grid_ms, _ = ctx.read_timing("grid")
    sort_ms, sorts = ctx.read_timing("sort")
    out_ms, _ = ctx.read_timing("output")
    init_ms, _ = ctx.read_timing("init")
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    n = cfg["n_steps"]
    job_s = (t1 - t0) / steps
    # Algorithmic bytes from the library's own count of the work of the timed
    # launches: particle-updates (with and without a drift) and mesh cells
    # read (each field mesh a launch gathers from; with several species on
    # their own re-sort cadence a plain launch may leave out the species a
    # fused re-sort pushed).
    kernels = {}
    wd, wk, mc = work_push
    kernels["k_push_f32" if cfg["precision"] == "fp32" else "k_push_f64"] = dict(
        ms=push_ms, launches=launches,
        bytes=wd * state_bytes(cfg, True) + wk * state_bytes(cfg, False) + mc * mesh_cell_bytes(cfg))
    if ps_launches:
        wd, _, mc = work_ps
        kernels["k_push_sort_f32"] = dict(ms=ps_ms, launches=ps_launches,
                                          bytes=wd * SORT_PUSH_STATE_BYTES + mc * mesh_cell_bytes(cfg))
    for k in kernels.values():
        k["avg_launch_ms"] = k["ms"] / k["launches"]
        k["bytes_per_launch"] = k["bytes"] / k["launches"]
        k["achieved_gbs"] = k["bytes_per_launch"] / (k["avg_launch_ms"] * 1e-3) / 1e9
        k["ms_per_job"] = k["ms"] / steps
        k["launches_per_job"] = k["launches"] / steps
    dominant = max(kernels, key=lambda name: kernels[name]["ms"])
    return dict(job_s=job_s, updates_per_s=n_total * n / job_s, kernels=kernels, dominant=dominant,
                push_ms=push_ms, launches=launches, avg_launch_ms=kernels[dominant]["avg_launch_ms"],
                achieved_gbs=kernels[dominant]["achieved_gbs"],
                grid_ms_per_job=grid_ms / steps, output_ms_per_job=out_ms / steps,
                init_ms_per_job=init_ms / steps, sort_ms_per_job=sort_ms / steps,
                sorts_per_job=sorts / steps, pk=pk, n_particles=n_total)


def traffic_from_profile(workload, kernel):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter
    summaries, if they were taken on the current push kernel source."""
    path = os.path.join(ROOT, "profiles", "push_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("push_source_sha256") != push_source_sha():
        return None
    return rec.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


def push_source_sha():
    """SHA-256 over the sources of the separable push kernel."""
    h = hashlib.sha256()
    for name in ("fdf_push.hip", "fdf_push_common.h"):
        with open(os.path.join(ROOT, "paper_2207_14256_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _cpu_worker(cfg, queue):
    try:
        queue.put(cpu_baseline(cfg))
    except Exception as exc:  # reported, never fatal for the GPU result
        queue.put({"error": repr(exc)})


_GRIDS = None


def _push_chunk(args):
    """Oracle push of one chunk of ids (runs in a forked worker that shares
    the parent's grids)."""
    import numpy as np
    from oracle import particles, pipeline, push
    cfg, ids, n_steps = args
    sp = cfg["species"][0]
    sched = pipeline.schedule(cfg)
    x0 = particles.positions_f64(sp["seed"], ids, cfg["box_mpc"])
    q0 = particles.momenta_f64(sp["seed"], ids)
    t0 = time.perf_counter()
    push.kdk(x0, q0, q0, sp["m"], sched, cfg["box_mpc"], lambda k: _GRIDS, 0, n_steps)
    return time.perf_counter() - t0, len(ids)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, per_core=32768, n_steps=40, max_workers=16):
    """The FP64 oracle (numpy) on a bounded sample of the same workload, run
    before the GPU legs: its own field and gradient grids at full mesh size,
    then per_core particles per core pushed through the first n_steps steps,
    on one core and on every host core available to the process (at most
    max_workers, forked workers sharing the grids)."""
    global _GRIDS
    import multiprocessing as mp
    import numpy as np
    from oracle import field, pipeline
    t0 = time.perf_counter()
    sched = pipeline.schedule(cfg)
    d0 = pipeline.delta0(cfg)
    _GRIDS = field.potential_grids(d0, cfg["box_mpc"], sched["a"][0], pipeline.model_of(cfg))
    t_setup = time.perf_counter() - t0
    log("cpu oracle: field + grids %.1f s" % t_setup)
    sp = cfg["species"][0]
    n_all = sp["n_side"] ** 3
    cores = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    stride = max(1, n_all // (per_core * cores))
    ids = np.arange(0, n_all, stride)[:per_core * cores]
    chunks = np.array_split(ids, cores)
    t_one, n_one = _push_chunk((cfg, chunks[0], n_steps))
    log("cpu oracle: 1 core %.1f s" % t_one)
    t1 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        parts = pool.map(_push_chunk, [(cfg, c, n_steps) for c in chunks])
    t_all = time.perf_counter() - t1
    log("cpu oracle: %d cores %.1f s" % (cores, t_all))
    _GRIDS = None
    n_done = sum(n for _, n in parts)
    return dict(value=n_done * n_steps / t_all, unit="particle-updates/s", cores=cores, kind="oracle",
                value_1core=n_one * n_steps / t_one, nproc=os.cpu_count(), cpu_model=_cpu_model(),
                sample="FP64 numpy oracle: %d of %d particles (every %d-th id) pushed through steps "
                       "0-%d of the %d-step schedule on the oracle's own %d^3 FP64 grids, split over "
                       "%d forked worker processes (%.1f s wall; the 1-core rate from one worker's "
                       "share alone, %.1f s); field + grid build %.1f s not in the rates; run before "
                       "the GPU legs" % (
                           n_done, n_all, stride, n_steps - 1, cfg["n_steps"], cfg["grid_n"], cores,
                           t_all, t_one, t_setup))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="tune the launch and sort policy first")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="start with a plain 4 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import multiprocessing as mp

    from paper_2207_14256_amd import workloads
    cfg = workloads.preset(args.workload)
    # the oracle (CPU only, numpy) runs first, in a spawned process that never
    # touches the GPU (so it may fork its workers), with the host to itself
    cpu = None
    if not args.no_cpu_baseline:
        mpc = mp.get_context("spawn")
        cpu_queue = mpc.Queue()
        cpu_proc = mpc.Process(target=_cpu_worker, args=(cfg, cpu_queue), daemon=False)
        cpu_proc.start()
        while cpu_proc.is_alive() and cpu_queue.empty():
            time.sleep(2)
        cpu = cpu_queue.get(timeout=120)
        cpu_proc.join(timeout=120)
        log("cpu oracle: %s" % {k: v for k, v in cpu.items() if k != "sample"})

    import numpy as np
    import torch
    from paper_2207_14256_amd import fastdf
    fastdf.load()
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    from paper_2207_14256_amd import autotune
    if args.autotune:
        autotune.autotune(cfg, log=log)
    tuning = autotune.cached_tuning(cfg)
    log("workload %s: precision %s, tuning %s" % (args.workload, cfg["precision"], tuning))
    main_leg = run_leg(cfg, args.steps, args.warmup, args.workload, tuning)
    log("%s: %.3e updates/s, %s %.3f ms/launch, %.0f GB/s" % (
        args.workload, main_leg["updates_per_s"], main_leg["dominant"], main_leg["avg_launch_ms"],
        main_leg["achieved_gbs"]))

    fp64 = None
    if not args.no_fp64_leg and cfg["precision"] == "fp32":
        cfg64 = workloads.preset(args.workload, precision="fp64")
        leg = run_leg(cfg64, max(1, args.steps - 1), 1, args.workload + "-fp64",
                      autotune.cached_tuning(cfg64))
        k32, p32, n32 = main_leg["pk"]
        k64, p64, n64 = leg["pk"]
        kn = np.pi * cfg["grid_n"] / cfg["box_mpc"]
        sel = (n64 > 0) & (k64 <= kn / 2)
        rel = np.abs(p32[sel] / p64[sel] - 1.0)
        fp64 = dict(updates_per_s=leg["updates_per_s"], ms_per_step=leg["job_s"] * 1e3,
                    push_ms_per_launch=leg["avg_launch_ms"], push_achieved_gbs=leg["achieved_gbs"],
                    push_roofline_frac=leg["achieved_gbs"] / PEAK_HBM_GBS,
                    push_ms_per_job=leg["push_ms"] / max(1, args.steps - 1),
                    sort_ms_per_job=leg["sort_ms_per_job"],
                    pk_rel_err_fp32_vs_fp64_max=float(rel.max()),
                    pk_rel_err_fp32_vs_fp64_rms=float(np.sqrt(np.mean(rel ** 2))),
                    pk_bins_compared="k <= k_N/2 (%d bins)" % int(sel.sum()))
        log("fp64 leg: %.3e updates/s, P(k) fp32/fp64 max rel diff %.2e" % (
            leg["updates_per_s"], rel.max()))

    traffic = traffic_from_profile(args.workload, main_leg["dominant"])
    out = {
        "metric": METRIC,
        "value": main_leg["updates_per_s"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["job_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg["precision"] == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: %d^3 neutrinos m=%g eV, %d^3 %s gradient mesh, L=%g Mpc, %d steps "
                        "z=%g->%g, %s" % (
                            args.workload, cfg["species"][0]["n_side"], cfg["species"][0]["m"],
                            cfg["grid_n"], "bf16" if cfg["precision"] == "fp32" else "f64",
                            cfg["box_mpc"], cfg["n_steps"], cfg["z_begin"], cfg["z_end"],
                            "FP32 push, uint32 fixed-point x, q = q0 + dq" if cfg["precision"] == "fp32"
                            else "FP64 push"),
            "particles": main_leg["n_particles"], "grid_n": cfg["grid_n"],
            "push_steps_per_job": cfg["n_steps"],
            "job": "field + sample + grid FFT + all push steps + weights + deposit/P(k)",
            "tuning": tuning,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": main_leg["achieved_gbs"],
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": main_leg["achieved_gbs"] / PEAK_HBM_GBS,
            "traffic": traffic,
            "kernel": main_leg["dominant"],
            "avg_launch_ms": main_leg["avg_launch_ms"],
            "algorithmic_bytes_per_launch": main_leg["kernels"][main_leg["dominant"]]["bytes_per_launch"],
            "mesh_padding_bytes_per_launch": mesh_padding_bytes(cfg),
        },
        "hbm_gbs": main_leg["achieved_gbs"],
        "kernels": {name: {k: v for k, v in rec.items() if k not in ("ms", "bytes")}
                    for name, rec in main_leg["kernels"].items()},
        "breakdown_ms_per_job": {
            "push": main_leg["push_ms"] / args.steps,
            "push_sort": main_leg["kernels"].get("k_push_sort_f32", {}).get("ms_per_job", 0.0),
            "sort": main_leg["sort_ms_per_job"],
            "sorts": main_leg["sorts_per_job"], "grid": main_leg["grid_ms_per_job"],
            "output": main_leg["output_ms_per_job"], "init": main_leg["init_ms_per_job"],
            "note": "push = plain push launches (one step each); push_sort = push launches that "
                    "also carry out a re-sort; sort = rank passes, scans and separate moves"},
        "fp64_leg": fp64,
        "speedup_vs_fp64": (main_leg["updates_per_s"] / fp64["updates_per_s"]) if fp64 else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
