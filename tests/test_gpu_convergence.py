"""Self-convergence of the density spectrum in Delta log a and in the mesh
size (sec. 4), through the C ABI: errors against the finest member of each
sequence must fall as the step or the mesh is refined."""
import numpy as np
import pytest

from paper_2207_14256_amd import convergence, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-case] %s" % msg, flush=True)


def _cfg(n_steps=20):
    cfg = workloads.small("c1", grid_n=32, n_side=32, n_steps=n_steps, box_mpc=1500.0, z_begin=1e6,
                          z_end=31.0, fixed_amp=True, precision="fp64")
    cfg["species"][0]["m"] = 0.1
    return cfg


def test_step_size_convergence():
    say("step-size convergence")
    res = convergence.step_study(_cfg(), factors=(1, 2, 4, 16), log=say)
    errs = [r["rms"] for r in res["runs"]]
    say("rms errors vs %d steps: %s" % (res["reference_steps"], errs))
    assert errs[0] > errs[1] > errs[2]
    # second-order leapfrog: about fourfold per halving once resolved
    assert errs[1] / errs[2] > 2.5


def test_mesh_size_convergence():
    say("mesh-size convergence")
    res = convergence.mesh_study(_cfg(n_steps=60), meshes=(16, 32, 64), log=say)
    errs = [r["rms"] for r in res["runs"]]
    say("rms errors vs mesh %d on analysis mesh %d: %s" % (res["reference_mesh"], res["analysis_mesh"], errs))
    assert errs[0] > errs[1]
