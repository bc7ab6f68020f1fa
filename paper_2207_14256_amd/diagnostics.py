"""History of the four acceleration terms of the exact geodesic equation over
a run (sec. 3.1, Fig. 2): the rms over one species of |eps grad psi|,
|(q^2/eps) grad phi|, |q (q . grad phi)/eps| and |q phidot| at a series of
schedule times, through the C ABI.

CLI: python -m paper_2207_14256_amd.diagnostics c3 --points 20 --out terms.json
"""
import json

import numpy as np

from . import fastdf, workloads

TERMS = ("newtonian", "q2_grad_phi", "q_q_grad_phi", "q_phidot")


def force_term_history(cfg, points=20, species=0):
    """Integrate the workload, sampling the terms at `points` + 1 evenly spaced
    schedule indices (the first and last included).  Returns a list of dicts
    with step, z and the four rms values."""
    ctx, fields, sids = fastdf.setup_workload(cfg)
    sched = ctx.read_schedule()
    n = cfg["n_steps"]
    marks = np.unique(np.linspace(0, n, points + 1).round().astype(int))
    out = []
    k = 0
    for m in marks:
        if m > k:
            ctx.step(int(m - k))
            k = int(m)
        rms = ctx.force_terms(sids[species])
        a = float(sched["a"][k])
        out.append(dict(step=k, z=1.0 / a - 1.0, **{t: float(v) for t, v in zip(TERMS, rms)}))
    ctx.close()
    return out


def main(argv=None):
    import argparse
    import sys

    import torch
    ap = argparse.ArgumentParser(description="rms of the acceleration terms of eq. releq over a run")
    ap.add_argument("workload")
    ap.add_argument("--points", type=int, default=20)
    ap.add_argument("--n-side", type=int, default=0)
    ap.add_argument("--mass", type=float, default=0.0)
    ap.add_argument("--model", choices=["poisson", "radmat"], default=None)
    ap.add_argument("--omega-r", type=float, default=None)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    cfg = workloads.preset(args.workload)
    cfg["species"] = cfg["species"][:1]
    if args.n_side:
        cfg["species"][0]["n_side"] = args.n_side
    if args.mass:
        cfg["species"][0]["m"] = args.mass
    if args.model:
        cfg["model"] = args.model
    if args.omega_r is not None:
        cfg["omega_r"] = args.omega_r
        cfg["omega_m"] = 1.0 - args.omega_r
    hist = force_term_history(cfg, args.points)
    text = json.dumps(dict(config={k: v for k, v in cfg.items() if k != "species"},
                           species=cfg["species"], history=hist), indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    for h in hist:
        print("z=%10.3g  " % h["z"] + "  ".join("%s %.3e" % (t, h[t]) for t in TERMS), file=sys.stderr)


if __name__ == "__main__":
    main()
