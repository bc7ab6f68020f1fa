"""Write c3_reduced_oracle.json: the FP64 oracle on the precision-form
workload at reduced size, the reference for the per-k-bin error statement of
the FP32 form.

Workload: the c3 physics (m = 0.1 eV, L = 1 Gpc, psi != phi, 1000 steps of
constant Delta log a from z = 1e9 to z = 0, field seed 1003, species seed
2030) with 64^3 particles on a 64^3 mesh.  Outputs: the binned energy-density
spectrum (sec. 4: cross spectrum of the even/odd halves, and the auto
spectrum) at z = 0, and the final positions, momenta and delta-f weights of
1024 sampled ids.  Only the oracle and the workload presets are used; the
particles are split over worker processes (each integrates its own ids on the
same grids, since particles are independent).

    python tests/golden/make_c3_reduced.py [--workers N]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import pipeline            # noqa: E402
from paper_2207_14256_amd import workloads   # noqa: E402

N_SIDE = 64
OUT = os.path.join(HERE, "c3_reduced_oracle.json")


def reduced_cfg():
    cfg = workloads.small("c3", grid_n=N_SIDE, n_side=N_SIDE, n_steps=1000)
    cfg["pk_bins"] = 32
    return cfg


def _run(ids):
    cfg = reduced_cfg()
    r = pipeline.run_particles(cfg, 0, ids)
    return ids, r["x"], r["q"], r["w"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    args = ap.parse_args()
    cfg = reduced_cfg()
    n = N_SIDE ** 3
    chunks = np.array_split(np.arange(n), 8 * args.workers)
    t0 = time.time()
    with mp.get_context("fork").Pool(args.workers) as pool:
        parts = pool.map(_run, chunks)
    x = np.concatenate([p[1] for p in parts])
    q = np.concatenate([p[2] for p in parts])
    w = np.concatenate([p[3] for p in parts])
    res = dict(x=x, q=q, w=w, sched=pipeline.schedule(cfg))
    (kc, pc, nc), _ = pipeline.density_spectrum(cfg, 0, res, "cross")
    (ka, pa, na), _ = pipeline.density_spectrum(cfg, 0, res, "auto")
    ids = workloads.sample_ids(n, 1024, seed=31)

    def lst(a):
        return [None if not np.isfinite(v) else float(v) for v in np.ravel(a)]

    rec = {
        "_source": "written by tests/golden/make_c3_reduced.py from the FP64 oracle only",
        "workload": "c3 physics at %d^3 particles on a %d^3 mesh: m=0.1 eV, L=1000 Mpc, slip 0.01, "
                    "1000 steps z=1e9->0, field seed 1003, species seed 2030" % (N_SIDE, N_SIDE),
        "grid_n": N_SIDE, "n_side": N_SIDE, "n_steps": 1000, "pk_bins": cfg["pk_bins"],
        "cross": {"k": lst(kc), "p": lst(pc), "nmodes": lst(nc)},
        "auto": {"k": lst(ka), "p": lst(pa), "nmodes": lst(na)},
        "sample_ids": [int(i) for i in ids],
        "x": lst(x[ids]), "q": lst(q[ids]), "w": lst(w[ids]),
        "oracle_seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, separators=(",", ":"))
    print("wrote %s (%.0f s)" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
