"""The spatial re-sort permutes the particle state only: results by id are
bit-identical for any sort cadence and tile size (GPU, through the C ABI)."""
import numpy as np
import pytest

from paper_2207_14256_amd import fastdf, workloads

pytestmark = pytest.mark.gpu


def _final_state(cfg, sort_every, tiles=0, steps=None):
    cfg = dict(cfg, sort_every=sort_every)
    ctx, fields, species = fastdf.setup_workload(cfg)
    if tiles:
        ctx.set_tuning(sort_tiles=tiles)
    ctx.step(cfg["n_steps"] if steps is None else steps)
    x, q = ctx.read_state(species[0])
    w = ctx.weights(species[0]).cpu().numpy()
    ctx.close()
    return x, q, w


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sort_cadence_invariance(prec):
    print("[gpu-case] sort cadence invariance %s" % prec, flush=True)
    cfg = workloads.small("c2", grid_n=32, n_side=29, n_steps=60, precision=prec,
                          box_mpc=600.0, z_begin=1e6, z_end=10.0)
    ref = _final_state(cfg, 0)
    for every, tiles in ((1, 0), (7, 0), (20, 4), (3, 16)):
        got = _final_state(cfg, every, tiles)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (every, tiles)


def test_sort_then_backward_walk():
    """Sorting in both directions of a forward-backward walk keeps ids aligned."""
    print("[gpu-case] sort + backward walk", flush=True)
    cfg = workloads.small("c2", grid_n=16, n_side=20, n_steps=30, precision="fp64",
                          box_mpc=500.0, z_begin=1e6, z_end=100.0, sort_every=4)
    ctx, fields, species = fastdf.setup_workload(cfg)
    x0, q0 = ctx.read_state(species[0])
    ctx.step(30)
    ctx.step(-30)
    x1, q1 = ctx.read_state(species[0])
    L = cfg["box_mpc"]
    d = (x1 - x0 + L / 2) % L - L / 2
    assert np.max(np.abs(d)) < 1e-10 * L
    assert np.max(np.abs(q1 - q0)) < 1e-10 * np.max(np.abs(q0))
    ctx.close()
