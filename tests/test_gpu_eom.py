"""The other equations of motion (sec. 3.1, 3.2, 5) on the GPU, through the C
ABI, against the oracle's explicit kick-drift-kick of the same equations.

Time-dependent potentials with gravitational slip (phi != psi, phi-dot != 0)
so that every term of every form acts."""
import numpy as np
import pytest

from oracle import field as ofield
from oracle import pipeline
from paper_2207_14256_amd import fastdf, workloads

pytestmark = pytest.mark.gpu

FORMS = ["exact", "canonical", "sr_newton", "simple_q", "newtonian"]


def say(msg):
    print("[gpu-case] %s" % msg, flush=True)


def periodic_diff(a, b, L):
    return (a - b + L / 2) % L - L / 2


def _cfg(eom, prec="fp64", **kw):
    base = dict(grid_n=16, n_side=13, n_steps=24, precision=prec, model="radmat", omega_m=0.9999,
                omega_r=1e-4, box_mpc=600.0, z_begin=1e5, z_end=30.0, slip_amp=0.3, slip_k=0.05,
                eom=eom)
    base.update(kw)
    return workloads.small("c2", **base)


def _run(cfg, steps=None):
    ctx, fields, species = fastdf.setup_workload(cfg)
    ctx.step(cfg["n_steps"] if steps is None else steps)
    x, q = ctx.read_state(species[0])
    w = ctx.weights(species[0]).cpu().numpy()
    return ctx, fields, species, x, q, w


@pytest.mark.parametrize("eom", FORMS)
def test_eom_parity_fp64(eom):
    say("eom %s fp64" % eom)
    cfg = _cfg(eom)
    ctx, fields, species, x, q, w = _run(cfg)
    ctx.close()
    n = cfg["species"][0]["n_side"] ** 3
    ref = pipeline.run_particles(cfg, 0, np.arange(n))
    L = cfg["box_mpc"]
    assert np.max(np.abs(periodic_diff(x, ref["x"], L))) < 1e-9 * L
    assert np.max(np.abs(q - ref["q"])) < 1e-9 * np.max(np.abs(ref["q"]))
    assert np.allclose(w, ref["w"], rtol=1e-5, atol=1e-7 * np.abs(ref["w"]).max())
    # the integration moved the momenta well beyond the tolerance
    assert np.median(np.linalg.norm(ref["q"] - ref["q0"], axis=1)) > 3e-5 * np.max(np.abs(ref["q"]))


def test_eom_poisson_exact_parity_fp64():
    """Static potentials, phi = psi: the phi-dot slot is an explicit zero."""
    say("eom exact poisson fp64")
    cfg = _cfg("exact", model="poisson", slip_amp=0.0, omega_m=1.0, omega_r=0.0, z_begin=1e4,
               z_end=30.0, n_side=11)
    ctx, fields, species, x, q, w = _run(cfg)
    ctx.close()
    ref = pipeline.run_particles(cfg, 0, np.arange(11 ** 3))
    L = cfg["box_mpc"]
    assert np.max(np.abs(periodic_diff(x, ref["x"], L))) < 1e-9 * L
    assert np.max(np.abs(q - ref["q"])) < 1e-9 * np.max(np.abs(ref["q"]))


@pytest.mark.parametrize("eom,quantities", [("exact", {9: ("phi", "psi")}),
                                            ("canonical", {7: ("psi",), 8: ("phi",)})])
def test_eom_potential_slots(eom, quantities):
    say("eom %s potential slots" % eom)
    cfg = _cfg(eom)
    ctx = fastdf.Context(cfg)
    fid = ctx.add_field(cfg["fields"][0])
    a = 2e-4
    ctx.build_potential_grids(fid, a)
    ref = ofield.potential_grids(pipeline.delta0(cfg), cfg["box_mpc"], a, pipeline.model_of(cfg),
                                 with_psi=True, with_phi=True)
    for qty, names in quantities.items():
        want = sum(ref[nm] for nm in names)
        got = ctx.read_grid(fid, qty)
        assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want)), qty
    with pytest.raises(fastdf.FastDFError):
        ctx.read_grid(fid, 8 if eom == "exact" else 9)     # not stored for this form
    ctx.close()


@pytest.mark.parametrize("eom", ["exact", "simple_q"])
def test_eom_fp32_error_statement(eom):
    """Precision form (fixed-point x, q = q0 + dq, bf16 mesh) against the FP64 oracle."""
    say("eom %s fp32" % eom)
    cfg = _cfg(eom, "fp32", grid_n=32, n_side=24, n_steps=40)
    ctx, fields, species, x, q, w = _run(cfg)
    ctx.close()
    ids = np.arange(24 ** 3)
    ref = pipeline.run_particles(cfg, 0, ids)
    L, G = cfg["box_mpc"], cfg["grid_n"]
    dx = periodic_diff(x, ref["x"], L) * (G / L)
    pos_rms = np.sqrt(np.mean(np.sum(dx ** 2, 1)))
    qrel = np.linalg.norm(q - ref["q"], axis=1) / np.linalg.norm(ref["q"] - ref["q0"], axis=1)
    say("fp32 %s: pos rms %.3e cells, kick rel err median %.3e" % (eom, pos_rms, np.median(qrel)))
    assert pos_rms < 1e-2
    assert np.median(qrel) < 1e-2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_eom_split_calls_bitwise(prec):
    """The half-kicks of a non-separable form are applied one after the other
    in either case, so step(a) + step(b) reproduces step(a + b) bit for bit."""
    say("eom split calls %s" % prec)
    cfg = _cfg("exact", prec)
    ctx, fields, species, x1, q1, w1 = _run(cfg)
    fastdf.setup_workload(cfg, ctx=ctx)
    ctx.step(9)
    ctx.step(cfg["n_steps"] - 9)
    x2, q2 = ctx.read_state(species[0])
    assert np.array_equal(x1, x2) and np.array_equal(q1, q2)
    for tuning in (dict(use_graph=1), dict(persistent_blocks=64, particles_per_thread=1)):
        fastdf.setup_workload(cfg, ctx=ctx)
        ctx.set_tuning(**tuning)
        ctx.step(cfg["n_steps"])
        x3, q3 = ctx.read_state(species[0])
        assert np.array_equal(x1, x3) and np.array_equal(q1, q3), tuning
        ctx.set_tuning(use_graph=0, persistent_blocks=0, particles_per_thread=4)
    ctx.close()


@pytest.mark.parametrize("n_steps", [60, 1142])
def test_separable_vs_exact_power_spectrum(n_steps):
    """Sec. 3.3: the non-symplectic integration of the exact equations and the
    separable scheme give nearly the same density spectra (the paper quotes
    about 1e-5 for its run; here the synthetic potentials give about 1e-4).
    1142 steps from z = 1e6 to 10 is the paper's Delta log a = 0.01; 60 steps
    is Delta log a = 0.19."""
    say("separable vs exact P(k), %d steps" % n_steps)
    out = {}
    for eom in ("separable", "exact"):
        cfg = _cfg(eom, grid_n=32, n_side=32, n_steps=n_steps, box_mpc=2000.0, z_begin=1e6, z_end=10.0,
                   slip_amp=0.0, species=[dict(field=0, m=0.1, n_side=32, seed=7)])
        ctx, fields, species, x, q, w = _run(cfg)
        out[eom] = ctx.power_spectrum(species, cfg["pk_bins"], "auto")
        ctx.close()
    k, ps, n = out["separable"]
    _, pe, _ = out["exact"]
    ok = n > 0
    rel = np.abs(pe[ok] / ps[ok] - 1)
    dloga = np.log((1 + 1e6) / (1 + 10.0)) / n_steps
    say("separable vs exact, dloga %.3f: max |dP/P| = %.3e, median %.3e" % (dloga, rel.max(), np.median(rel)))
    # recorded: median 8.7e-5 / 9.9e-5 and max 6.2e-4 / 6.8e-4 (1142 / 60
    # steps); the paper quotes about 1e-5 for its own run
    assert np.median(rel) < 3e-4 and rel.max() < 2e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_force_terms_parity(prec):
    """Fig. 2 diagnostic: rms of the four terms of eq. releq over the species,
    at the start and after the run, against the oracle's at its own state."""
    say("force terms %s" % prec)
    cfg = _cfg("separable", prec)
    ctx, fields, species = fastdf.setup_workload(cfg)
    start = ctx.force_terms(species[0])
    ctx.step(cfg["n_steps"])
    end = ctx.force_terms(species[0])
    ctx.close()
    n = cfg["species"][0]["n_side"] ** 3
    ref = pipeline.run_particles(cfg, 0, np.arange(n))
    sched = pipeline.schedule(cfg)
    grids = pipeline.grids_provider(cfg, pipeline.delta0(cfg), sched)
    m, L = cfg["species"][0]["m"], cfg["box_mpc"]
    from oracle import push as opush
    r0 = opush.force_term_rms(grids(0), ref["x0"], ref["q0"], m, sched["a"][0], L)
    r1 = opush.force_term_rms(grids(cfg["n_steps"]), ref["x"], ref["q"], m, sched["a"][-1], L)
    tol = 1e-9 if prec == "fp64" else 1e-2
    say("terms start %s / %s, end %s / %s" % (start, r0, end, r1))
    assert np.all(r0 > 0) and np.all(r1 > 0)
    assert np.allclose(start, r0, rtol=tol) and np.allclose(end, r1, rtol=tol)
