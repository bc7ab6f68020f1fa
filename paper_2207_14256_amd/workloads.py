"""Seeded synthetic workloads shared by the tests, the benchmark and smoke().

This module holds parameters and seeds only (plus small hand-placed particle
sets built with numpy's own generator for pin tests); none of the method's
arithmetic lives here.  Both the HIP path and the CPU oracle receive these
values as inputs.

Presets c1-c5 follow the five workload descriptions of the benchmark
specification: c1 32^3 FP64 EdS; c2 256^3 FP64 with gravitational slip;
c3 512^3 precision form; c4 batched species and seeds; c5 1024^3 scale run.
Cosmology: h = 0.7, Einstein-de Sitter background (Omega_m = 1), BBKS shape
Gamma = 0.2, n_s = 0.965, sigma_8 = 0.8.  Field seed = 1000 + preset index,
species seed = 2000 + 10 * preset index + species index.  sort_every enables
the spatial re-sort; sort_cells > 0 replaces the fixed cadence by the adaptive
one (re-sort after that many cells of typical drift).
"""
import copy

import numpy as np

BASE = dict(h=0.7, omega_m=1.0, omega_r=0.0, omega_l=0.0, ns=0.965, sigma8=0.8,
            gamma=0.2, model="poisson", slip_amp=0.0, slip_k=1.0,
            fixed_amp=False, pk_bins=64, sort_every=0, sort_cells=0.0, pre_ic=False)


def _preset(idx, **kw):
    cfg = copy.deepcopy(BASE)
    cfg.update(kw)
    cfg["preset"] = idx
    return cfg


PRESETS = {
    "c1": _preset(1, grid_n=32, box_mpc=512.0, z_begin=1e6, z_end=31.0, n_steps=50,
                  precision="fp64", fields=[1001],
                  species=[dict(field=0, m=0.1, n_side=32, seed=2010)]),
    "c2": _preset(2, grid_n=256, box_mpc=1000.0, z_begin=1e9, z_end=31.0, n_steps=500,
                  precision="fp64", slip_amp=0.01, slip_k=1.0, fields=[1002],
                  species=[dict(field=0, m=0.06, n_side=256, seed=2020)]),
    "c3": _preset(3, grid_n=512, box_mpc=1000.0, z_begin=1e9, z_end=0.0, n_steps=1000,
                  precision="fp32", slip_amp=0.01, slip_k=1.0, fields=[1003],
                  species=[dict(field=0, m=0.1, n_side=512, seed=2030)], sort_every=20,
                  sort_cells=2.0),
    "c4": _preset(4, grid_n=256, box_mpc=768.0, z_begin=1e9, z_end=31.0, n_steps=300,
                  precision="fp32", slip_amp=0.01, slip_k=1.0,
                  fields=[1004 + 100 * s for s in range(17)],
                  species=([dict(field=0, m=0.005, n_side=128, seed=2040),
                            dict(field=0, m=0.00995, n_side=256, seed=2041),
                            dict(field=0, m=0.0502, n_side=384, seed=2042)]
                           + [dict(field=s, m=0.05, n_side=128, seed=2043 + s)
                              for s in range(1, 17)]), sort_every=20, sort_cells=2.0),
    "c5": _preset(5, grid_n=512, box_mpc=2000.0, z_begin=1e9, z_end=0.0, n_steps=1000,
                  precision="fp32", slip_amp=0.01, slip_k=1.0, fields=[1005],
                  species=[dict(field=0, m=0.15, n_side=1024, seed=2050)], sort_every=20),
}


def preset(name, **overrides):
    """A deep copy of a preset with selected keys replaced."""
    cfg = copy.deepcopy(PRESETS[name])
    cfg.update(overrides)
    return cfg


def small(name="c1", grid_n=16, n_side=16, n_steps=50, **kw):
    """A reduced copy of a preset for quick parity cases (same physics)."""
    cfg = preset(name, grid_n=grid_n, n_steps=n_steps, **kw)
    for sp in cfg["species"]:
        sp["n_side"] = n_side
    return cfg


def n_particles(species):
    return int(species.get("n", species["n_side"] ** 3))


def sample_ids(n_total, count, seed=12345):
    """A sorted random subset of particle ids (numpy generator, seeded)."""
    rng = np.random.default_rng(seed)
    count = min(count, n_total)
    return np.sort(rng.choice(n_total, size=count, replace=False)).astype(np.int64)


def hand_placed(count, box_mpc, seed=7, q_scale=5e-4):
    """Hand-placed test particles: positions (uint32 lattice) and binary32 momenta."""
    rng = np.random.default_rng(seed)
    xu = rng.integers(0, 2 ** 32, size=(count, 3), dtype=np.uint64).astype(np.uint32)
    q = (rng.normal(size=(count, 3)) * q_scale).astype(np.float32)
    return xu, q
