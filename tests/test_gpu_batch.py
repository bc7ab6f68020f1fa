"""Batched species and seeds in one launch per step, persistent grids and
hipGraph replay (GPU, through the C ABI).

Every species is advanced by the same per-particle code whatever else shares
the launch, so a batched run must reproduce single-species runs bit for bit,
and so must the persistent-grid and graph-replay variants."""
import numpy as np
import pytest

from oracle import pipeline
from paper_2207_14256_amd import fastdf, workloads

pytestmark = pytest.mark.gpu


def _batched_cfg(prec):
    # three masses on field 0 (uneven counts) plus two independent seeds, c4-like
    cfg = workloads.small("c4", grid_n=32, n_side=0, n_steps=40, precision=prec, box_mpc=768.0,
                          z_begin=1e9, z_end=31.0, sort_every=4, sort_cells=0.0)
    cfg["fields"] = [1004, 1104, 1204]
    cfg["species"] = [dict(field=0, m=0.005, n_side=9, seed=2040),
                      dict(field=0, m=0.00995, n_side=17, seed=2041),
                      dict(field=0, m=0.0502, n_side=23, seed=2042),
                      dict(field=1, m=0.05, n_side=11, seed=2044),
                      dict(field=2, m=0.05, n_side=11, seed=2045)]
    return cfg


def _states(ctx, species):
    out = []
    for s in species:
        x, q = ctx.read_state(s)
        out.append((x, q, ctx.weights(s).cpu().numpy()))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_equals_single_species(prec):
    print("[gpu-case] batched vs single %s" % prec, flush=True)
    cfg = _batched_cfg(prec)
    ctx, fields, species = fastdf.setup_workload(cfg)
    ctx.step(cfg["n_steps"])
    batched = _states(ctx, species)
    ctx.close()
    for i, sp in enumerate(cfg["species"]):
        one = dict(cfg, fields=[cfg["fields"][sp["field"]]], species=[dict(sp, field=0)])
        c1, _, s1 = fastdf.setup_workload(one)
        c1.step(one["n_steps"])
        single = _states(c1, s1)[0]
        c1.close()
        for a, b in zip(batched[i], single):
            assert np.array_equal(a, b), (prec, i)


def test_batched_parity_with_oracle():
    """Two species of the batch (different fields and masses) against the oracle."""
    print("[gpu-case] batched parity fp64", flush=True)
    cfg = _batched_cfg("fp64")
    ctx, fields, species = fastdf.setup_workload(cfg)
    ctx.step(cfg["n_steps"])
    L = cfg["box_mpc"]
    for i in (1, 3):
        x, q = ctx.read_state(species[i])
        n = cfg["species"][i]["n_side"] ** 3
        ref = pipeline.run_particles(cfg, i, np.arange(n))
        d = (x - ref["x"] + L / 2) % L - L / 2
        assert np.max(np.abs(d)) < 1e-5 * L
        assert np.max(np.abs(q - ref["q"])) < 1e-9 * np.max(np.abs(ref["q"]))
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_persistent_and_graph_modes_bitwise(prec):
    print("[gpu-case] persistent + graph %s" % prec, flush=True)
    cfg = _batched_cfg(prec)
    ctx, fields, species = fastdf.setup_workload(cfg)
    ctx.step(15)                       # same call split as below: the seam's two
    ctx.step(cfg["n_steps"] - 15)      # half-kicks are applied separately
    ref = _states(ctx, species)
    for tuning in (dict(persistent_blocks=64), dict(use_graph=1), dict(use_graph=1, persistent_blocks=2048),
                   dict(particles_per_thread=1), dict(particles_per_thread=8, use_graph=1)):
        fastdf.setup_workload(cfg, ctx=ctx)
        ctx.set_tuning(**tuning)
        ctx.step(15)
        ctx.step(cfg["n_steps"] - 15)
        got = _states(ctx, species)
        for a, b in zip(got, ref):
            for u, v in zip(a, b):
                assert np.array_equal(u, v), tuning
        # replay: the same layout and schedule again reuses the captured graphs
        fastdf.setup_workload(cfg, ctx=ctx)
        ctx.step(15)
        ctx.step(cfg["n_steps"] - 15)
        again = _states(ctx, species)
        for a, b in zip(again, ref):
            for u, v in zip(a, b):
                assert np.array_equal(u, v), ("replay", tuning)
        ctx.set_tuning(persistent_blocks=0, use_graph=0, particles_per_thread=4)
    ctx.close()
