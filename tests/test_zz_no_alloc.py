"""The no-allocation spectrum entry point (fdf_power_spectrum_noalloc)
against fdf_power_spectrum on the same context, through the C ABI: two calls
in a row, the second on a smaller input, both quantities, both arithmetic
forms.  FP32 form: the fixed-point deposit makes both entry points bit-equal;
FP64 form: the float64 atomics' order leaves rounding-level differences."""
import sys

import numpy as np
import pytest

from paper_2207_14256_amd import fastdf, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def _check(ctx, species, nbins, mode, quantity, analysis_n, out, exact):
    k, p, nm = ctx.power_spectrum(species, nbins, mode, quantity, analysis_n=analysis_n)
    ctx.power_spectrum_noalloc(species, nbins, out, mode, quantity, analysis_n)
    ctx.sync()
    o = out.cpu().numpy()
    k2, p2, n2 = o[:nbins], o[nbins:2 * nbins], o[2 * nbins:3 * nbins]
    assert np.array_equal(nm, n2)
    ok = nm > 0
    assert np.all(np.isnan(k2[~ok])) and np.all(np.isnan(p2[~ok]))
    assert np.array_equal(k[ok], k2[ok])
    if exact:
        assert np.array_equal(p[ok], p2[ok])
    else:
        assert np.allclose(p[ok], p2[ok], rtol=1e-12, atol=1e-14 * np.abs(p[ok]).max())


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_spectrum_matches_workspace_spectrum(prec):
    import torch
    torch.cuda.set_device(0)
    say("no-alloc spectrum %s" % prec)
    cfg = workloads.small("c4", grid_n=64, n_side=0, n_steps=60, precision=prec, box_mpc=768.0,
                          z_begin=1e9, z_end=31.0, sort_every=4, sort_cells=0.0)
    cfg["fields"] = [1004]
    cfg["species"] = [dict(field=0, m=0.005, n_side=24, seed=2040),
                      dict(field=0, m=0.0502, n_side=31, seed=2042)]
    ctx, fields, species = fastdf.setup_workload(cfg)
    ctx.step(cfg["n_steps"])
    out = torch.full((3 * 40,), 7.0, dtype=torch.float64, device="cuda")
    exact = prec == "fp32"
    # first call: both species, the 64^3 analysis mesh; second: one species, 16^3
    _check(ctx, species, 40, "cross", "density", 64, out, exact)
    _check(ctx, species[:1], 12, "cross", "density", 16, out, exact)
    _check(ctx, species, 20, "auto", "momentum", 32, out, exact)
    _check(ctx, species[1:], 10, "cross", "momentum", 8, out, exact)
    ctx.close()


def test_noalloc_refuses_large_mesh():
    import torch
    torch.cuda.set_device(0)
    say("no-alloc refusal")
    cfg = workloads.small("c2", grid_n=128, n_side=8, n_steps=2, precision="fp32", box_mpc=1000.0,
                          z_begin=1e6, z_end=1e5)
    ctx, fields, species = fastdf.setup_workload(cfg)
    ctx.step(cfg["n_steps"])
    out = torch.zeros(3 * 8, dtype=torch.float64, device="cuda")
    with pytest.raises(fastdf.FastDFError, match="at most 64"):
        ctx.power_spectrum_noalloc(species, 8, out)
    with pytest.raises(fastdf.FastDFError, match="at most 64"):
        ctx.power_spectrum_noalloc(species, 8, out, analysis_n=128)
    ctx.power_spectrum_noalloc(species, 8, out, analysis_n=64)   # within the limit
    ctx.sync()
    assert np.isfinite(out.cpu().numpy()[16:]).all()
    ctx.close()
