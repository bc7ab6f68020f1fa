"""Self-convergence of the neutrino spectra in the step size and the mesh size
(sec. 4: the two parameters that set precision and speed, Delta log a and the
potential mesh M).

Without a Boltzmann code to compare against, each sequence is compared with
its own finest member:

  steps: the same workload with n, 2n, 4n, ... steps (Delta log a halved each
         time); the leapfrog is second order, so the error should fall about
         fourfold per halving;
  mesh:  the same random field on meshes M/4, M/2, M (the coarse fields are
         the fine field's modes below their Nyquist frequency), with every
         spectrum estimated on the coarsest mesh so that only the force
         resolution differs.

Errors are max and rms of |P/P_finest - 1| over bins with k <= k_N / 2 of the
analysis mesh (k_N = pi M / L).  Runs go through the C ABI like any other.

CLI: python -m paper_2207_14256_amd.convergence c1 --out result.json
"""
import json
import time

import numpy as np

from . import fastdf, workloads


def truncate_field(delta_k, G_coarse):
    """Modes of a half-complex (G, G, G/2 + 1) field with |n_a| < G_coarse/2,
    as a (G_coarse, G_coarse, G_coarse/2 + 1) field; Nyquist entries zero."""
    G = delta_k.shape[0]
    Gc = int(G_coarse)
    n = np.arange(Gc)
    signed = np.where(n < Gc // 2, n, n - Gc)
    src = signed % G
    out = delta_k[np.ix_(src, src, np.arange(Gc // 2 + 1))].copy()
    out[Gc // 2, :, :] = 0
    out[:, Gc // 2, :] = 0
    out[:, :, Gc // 2] = 0
    return out


def run_spectrum(cfg, field=None, analysis_n=0, quantity="density", mode="cross"):
    """Integrate the workload and return (k, P, modes, seconds); field, when
    given, replaces the workload's first seeded field."""
    import torch
    ctx = fastdf.Context(cfg)
    if field is None:
        fids = [ctx.add_field(s, cfg.get("fixed_amp", False)) for s in cfg["fields"]]
    else:
        fids = [ctx.set_field(field)]
    sids = [ctx.init_species(fids[sp["field"]], sp["m"], workloads.n_particles(sp), sp["seed"],
                             cfg.get("pre_ic", False)) for sp in cfg["species"]]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(cfg["n_steps"])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    k, p, nm = ctx.power_spectrum(sids, cfg["pk_bins"], mode, quantity, analysis_n)
    ctx.close()
    return k, p, nm, secs


def _errors(k, p, ref, kmax):
    sel = np.isfinite(p) & np.isfinite(ref) & (k <= kmax) & (ref != 0)
    rel = np.abs(p[sel] / ref[sel] - 1.0)
    return dict(max=float(rel.max()), rms=float(np.sqrt(np.mean(rel ** 2))), bins=int(sel.sum()))


def step_study(cfg, factors=(1, 2, 4, 8), quantity="density", log=print):
    """Spectra at n_steps * f for each f; errors against the largest f."""
    runs = []
    for f in factors:
        c = dict(cfg, n_steps=int(cfg["n_steps"] * f))
        k, p, nm, secs = run_spectrum(c, quantity=quantity)
        runs.append(dict(n_steps=c["n_steps"], k=k, p=p, seconds=secs))
        log("[convergence] steps %d: %.2f s" % (c["n_steps"], secs))
    kmax = 0.5 * np.pi * cfg["grid_n"] / cfg["box_mpc"]
    ref = runs[-1]["p"]
    out = []
    for r in runs[:-1]:
        e = _errors(r["k"], r["p"], ref, kmax)
        out.append(dict(n_steps=r["n_steps"], seconds=r["seconds"], **e))
    return dict(kind="steps", quantity=quantity, reference_steps=runs[-1]["n_steps"], k_max=kmax,
                runs=out, k=runs[-1]["k"].tolist(), p_reference=ref.tolist())


def mesh_study(cfg, meshes=None, quantity="density", log=print):
    """Spectra on meshes M/4, M/2, M with one random field; all estimated on
    the coarsest mesh; errors against the finest mesh."""
    G = cfg["grid_n"]
    meshes = sorted(meshes or (G // 4, G // 2, G))
    Gmax, Ga = meshes[-1], meshes[0]
    fine = dict(cfg, grid_n=Gmax)
    ctx = fastdf.Context(fine)
    fid = ctx.add_field(cfg["fields"][0], cfg.get("fixed_amp", False))
    delta = ctx.read_field(fid)
    ctx.close()
    runs = []
    for M in meshes:
        c = dict(cfg, grid_n=M, fields=[cfg["fields"][0]],
                 species=[dict(sp, field=0) for sp in cfg["species"]])
        field = delta if M == Gmax else truncate_field(delta, M)
        k, p, nm, secs = run_spectrum(c, field=field, analysis_n=Ga, quantity=quantity)
        runs.append(dict(mesh=M, k=k, p=p, seconds=secs))
        log("[convergence] mesh %d: %.2f s" % (M, secs))
    kmax = 0.5 * np.pi * Ga / cfg["box_mpc"]
    ref = runs[-1]["p"]
    out = []
    for r in runs[:-1]:
        e = _errors(r["k"], r["p"], ref, kmax)
        out.append(dict(mesh=r["mesh"], seconds=r["seconds"], **e))
    return dict(kind="mesh", quantity=quantity, reference_mesh=Gmax, analysis_mesh=Ga, k_max=kmax,
                runs=out, k=runs[-1]["k"].tolist(), p_reference=ref.tolist())


def main(argv=None):
    import argparse
    import sys

    import torch
    ap = argparse.ArgumentParser(description="step-size and mesh-size self-convergence of P(k)")
    ap.add_argument("workload", help="preset name (c1 ... c5)")
    ap.add_argument("--n-side", type=int, default=0, help="particles per side (0: the preset's)")
    ap.add_argument("--grid-n", type=int, default=0, help="finest mesh (0: the preset's)")
    ap.add_argument("--box", type=float, default=0.0, help="box side [Mpc] (0: the preset's)")
    ap.add_argument("--z-end", type=float, default=None)
    ap.add_argument("--dloga", type=float, default=0.0, help="coarsest step in log a (0: the preset's)")
    ap.add_argument("--factors", default="1,2,4,8")
    ap.add_argument("--mass", type=float, default=0.0)
    ap.add_argument("--quantity", default="density", choices=["density", "momentum"])
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    kw = {}
    if args.grid_n:
        kw["grid_n"] = args.grid_n
    if args.box:
        kw["box_mpc"] = args.box
    if args.z_end is not None:
        kw["z_end"] = args.z_end
    cfg = workloads.preset(args.workload, **kw)
    cfg["species"] = cfg["species"][:1]
    if args.n_side:
        cfg["species"][0]["n_side"] = args.n_side
    if args.mass:
        cfg["species"][0]["m"] = args.mass
    cfg["fixed_amp"] = True
    if args.dloga:
        cfg["n_steps"] = max(1, int(round(np.log((1 + cfg["z_begin"]) / (1 + cfg["z_end"])) / args.dloga)))
    log = lambda m: print(m, file=sys.stderr, flush=True)
    factors = tuple(int(f) for f in args.factors.split(","))
    res = dict(config={k: v for k, v in cfg.items() if k != "species"}, species=cfg["species"],
               steps=step_study(cfg, factors, args.quantity, log),
               mesh=mesh_study(cfg, quantity=args.quantity, log=log))
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    for study in ("steps", "mesh"):
        for r in res[study]["runs"]:
            print(study, {k: v for k, v in r.items()})


if __name__ == "__main__":
    main()
