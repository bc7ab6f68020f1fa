"""GPU parity of the total density spectrum over several species and of the
pre-initial transform's dipole, against the FP64 CPU oracle (through the C ABI).

Total contrast (sec. 2.2 eq. empirical_rho per species, sec. 4 spectra): the
species of one field enter with weights <eps>_s / sum <eps>; the library
refuses species of different fields.  Pre-initial conditions (sec. 2.1 eq.
transform): a late start, where k tau >> 1, makes the dipole term
grad(nabla^-2 theta) the bulk of the transform, so the comparison sees it
rather than the binary32 rounding of q."""
import sys

import numpy as np
import pytest

from oracle import background, pipeline
from paper_2207_14256_amd import fastdf, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    torch.cuda.set_device(0)
    fastdf.load()
    yield
    torch.cuda.synchronize()


def _three_mass_cfg(prec):
    # the normal-hierarchy masses of the batched workload on one field, uneven
    # counts (one odd), plus an independent seed on a second field
    cfg = workloads.small("c4", grid_n=32, n_side=0, n_steps=30, precision=prec, box_mpc=768.0,
                          z_begin=1e9, z_end=31.0)
    cfg["fields"] = [1004, 1104]
    cfg["species"] = [dict(field=0, m=0.005, n_side=12, seed=2040),
                      dict(field=0, m=0.00995, n_side=17, seed=2041),
                      dict(field=0, m=0.0502, n_side=20, seed=2042),
                      dict(field=1, m=0.05, n_side=10, seed=2044)]
    cfg["pk_bins"] = 24
    return cfg


# measured: FP32 form against the FP64 oracle, max over bins with modes
FP32_TOTAL_PK_BOUND = 2e-2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_total_density_spectrum_parity(prec):
    say("total density spectrum, three masses, %s" % prec)
    cfg = _three_mass_cfg(prec)
    ctx, fields, species = fastdf.setup_workload(cfg)
    ctx.step(cfg["n_steps"])
    results = [pipeline.run_particles(cfg, i, np.arange(workloads.n_particles(cfg["species"][i])))
               for i in range(3)]
    for mode in ("cross", "auto"):
        k, p, nm = ctx.power_spectrum(species[:3], cfg["pk_bins"], mode)
        (kr, pr, nr), _ = pipeline.total_density_spectrum(cfg, [0, 1, 2], results, mode)
        assert np.array_equal(nm, nr)
        ok = nr > 0
        assert np.allclose(k[ok], kr[ok], rtol=1e-12)
        assert np.all(np.isnan(p[~ok]))
        rel = np.abs(p[ok] - pr[ok]) / np.abs(pr[ok]).max()
        say("%s %s: max |dP|/max|P| = %.3e" % (prec, mode, rel.max()))
        if prec == "fp64":
            assert np.allclose(p[ok], pr[ok], rtol=1e-6, atol=1e-9 * np.abs(pr[ok]).max())
        else:
            assert rel.max() < FP32_TOTAL_PK_BOUND
    # one species alone is that species' own spectrum, and the order of the
    # list does not matter beyond rounding
    k1, p1, _ = ctx.power_spectrum([species[2], species[0], species[1]], cfg["pk_bins"], "cross")
    k0, p0, _ = ctx.power_spectrum(species[:3], cfg["pk_bins"], "cross")
    ok = np.isfinite(p0)
    assert np.allclose(p1[ok], p0[ok], rtol=1e-5, atol=1e-9 * np.abs(p0[ok]).max())
    # species of different fields, or listed twice, are refused
    with pytest.raises(fastdf.FastDFError):
        ctx.power_spectrum([species[0], species[3]], cfg["pk_bins"], "cross")
    with pytest.raises(fastdf.FastDFError):
        ctx.power_spectrum([species[1], species[1]], cfg["pk_bins"], "cross")
    ctx.close()


def test_pre_initial_dipole_parity_late_start():
    """eq. transform at z = 100 in a 100 Mpc box (a short schedule to z = 95,
    whose drifts stay below half the box): the transform shift q0 - p is
    mostly the dipole (omega eps / nu) grad(nabla^-2 theta), and it must match
    the oracle's (pinned against -(tau/2) grad psi) within the binary32
    rounding of q0."""
    say("pre-IC dipole, late start fp64")
    cfg = workloads.small("c2", grid_n=16, n_side=16, n_steps=4, precision="fp64", box_mpc=100.0,
                          z_begin=100.0, z_end=95.0, pre_ic=True, slip_amp=0.0)
    cfg["species"][0]["m"] = 0.02
    ctx, fields, species = fastdf.setup_workload(cfg)
    q0 = ctx.read_state(species[0])[1]
    ids = np.arange(16 ** 3)
    ref = pipeline.run_particles(cfg, 0, ids, k_end=0)
    shift_ref = ref["q"] - ref["p"]
    shift_gpu = q0 - ref["p"]
    # the monopole part of the shift is at most |p| max|delta| / nu; the
    # dipole must dominate it here (k tau >> 1)
    sched = pipeline.schedule(cfg)
    a_i = sched["a"][0]
    tau_i = background.conformal_time(a_i, cfg["h"], cfg["omega_m"])
    d_grid, _ = pipeline.super_horizon_grids(cfg, pipeline.delta0(cfg), a_i, tau_i)
    mono = np.abs(ref["p"]).max() * np.abs(d_grid).max() / 4.0
    assert np.abs(shift_ref).max() > 10 * mono
    ulp = np.abs(ref["q"]).max() * 2.0 ** -23
    assert np.max(np.abs(shift_gpu - shift_ref)) <= ulp
    w0 = ctx.weights(species[0]).cpu().numpy()
    assert np.allclose(w0, ref["w"], rtol=1e-3, atol=1e-3 * np.abs(ref["w"]).max())
    ctx.close()


def test_fp32_spectra_bit_identical_across_runs_and_launch_shapes():
    """The FP32 form's deposit and binning sum in fixed point, so a spectrum
    does not depend on the order of the additions: repeated runs, and runs
    with another launch shape or re-sort cadence (which permute the particles
    but leave every particle's state bit-identical), give the same bits.  The
    never-sorted run keeps the particles in their random sampling order, so
    each deposit block touches more distinct cells than its LDS table holds
    and part of its contributions take the direct global atomics."""
    say("fp32 spectra bit-identical")
    cfg = workloads.small("c3", grid_n=32, n_side=40, n_steps=200, z_begin=1e9, z_end=3.0,
                          sort_every=4, sort_cells=0.0)
    out = []
    for tuning in (dict(particles_per_thread=4), dict(particles_per_thread=4),
                   dict(particles_per_thread=1, sort_every=7, push_waves=3),
                   dict(particles_per_thread=8, sort_every=0)):
        ctx, fields, species = fastdf.setup_workload(cfg)
        ctx.set_tuning(**tuning)
        ctx.step(cfg["n_steps"])
        res = [ctx.power_spectrum(species, 20, mode, quantity)
               for mode in ("cross", "auto") for quantity in ("density", "momentum")]
        ctx.close()
        out.append(res)
    for other in out[1:]:
        for (k0, p0, n0), (k1, p1, n1) in zip(out[0], other):
            assert np.array_equal(n0, n1) and np.array_equal(k0[n0 > 0], k1[n1 > 0])
            assert np.array_equal(p0[n0 > 0], p1[n1 > 0])
