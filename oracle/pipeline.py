"""End-to-end oracle runs of a workload (test infrastructure only).

A workload is a plain dict of parameters and seeds (see the workload presets
of the product package); this module composes the oracle's steps in the order
of the method: schedule -> field -> potential grids -> sample -> push ->
weights -> density -> P(k).  Any subset of particle ids can be integrated,
because particles are independent given the grids (sec. 2.1, last paragraph).
"""
import os

import numpy as np
from scipy import fft as sfft

from . import background, field, particles, push, stats


def cosmo_args(cfg):
    return (cfg["h"], cfg["omega_m"], cfg.get("omega_r", 0.0), cfg.get("omega_l", 0.0))


def model_of(cfg):
    return dict(kind=cfg["model"], h=cfg["h"], omega_m=cfg["omega_m"],
                omega_r=cfg.get("omega_r", 0.0), omega_l=cfg.get("omega_l", 0.0),
                slip_amp=cfg.get("slip_amp", 0.0), slip_k=cfg.get("slip_k", 1.0))


def schedule(cfg):
    return background.step_schedule(cfg["z_begin"], cfg["z_end"], cfg["n_steps"],
                                    *cosmo_args(cfg))


def amplitude(cfg):
    return field.power_amplitude(cfg["sigma8"], cfg["ns"], cfg["gamma"], cfg["h"])


def delta0(cfg, field_index=0):
    return field.gaussian_field(cfg["grid_n"], cfg["box_mpc"], cfg["fields"][field_index],
                                amplitude(cfg), cfg["ns"], cfg["gamma"], cfg["h"],
                                cfg.get("fixed_amp", False))


def superstep_anchors(cfg, sched, tol):
    """Super-steps of sec. 2.1 (last paragraph): potential grids are computed
    only when the transfer functions have changed by more than tol since the
    last computed set.  Starting at the first time of the schedule, the next
    anchor is the first schedule time a_k with max |T(k, a_k)/T(k, a_anchor) - 1|
    > tol over phi and psi; the last time of the schedule closes the list.
    Returns schedule indices."""
    model = model_of(cfg)
    ks = np.array([1e-3, 1e-2, 0.1, 1.0])
    a = sched["a"]

    def transfers(ai):
        t_phi, t_psi, _ = field.potential_transfers(ks, ai, model)
        return np.concatenate([t_phi, t_psi])

    anchors = [0]
    ref = transfers(a[0])
    for k in range(1, len(a)):
        cur = transfers(a[k])
        if np.max(np.abs(cur / ref - 1.0)) > tol:
            anchors.append(k)
            ref = cur
    if anchors[-1] != len(a) - 1:
        anchors.append(len(a) - 1)
    return anchors


def grids_provider(cfg, d0, sched, with_psi=False, with_phi=False):
    """grids_at(k) for the schedule.  Time-independent potentials: one build.
    Time-dependent potentials: a rebuild at every a_k, or, with
    cfg['superstep_tol'] > 0, the super-step scheme of sec. 2.1: grids at the
    anchors and, in between, linear interpolation in a,
        G(a_k) = (1 - t) G(a_A) + t G(a_B),  t = (a_k - a_A) / (a_B - a_A)."""
    L = cfg["box_mpc"]
    model = model_of(cfg)
    if model["kind"] == "poisson":
        g = field.potential_grids(d0, L, sched["a"][0], model, with_psi, with_phi)
        return lambda k: g
    cache = {}

    def build(k):
        if k not in cache:
            if len(cache) > 3:
                cache.clear()
            cache[k] = field.potential_grids(d0, L, sched["a"][k], model, with_psi, with_phi)
        return cache[k]

    tol = cfg.get("superstep_tol", 0.0)
    if tol <= 0:
        return build
    anchors = superstep_anchors(cfg, sched, tol)
    a = sched["a"]

    def at(k):
        i = max(j for j in range(len(anchors) - 1) if anchors[j] <= k) if k < anchors[-1] else len(anchors) - 2
        kA, kB = anchors[i], anchors[i + 1]
        t = (a[k] - a[kA]) / (a[kB] - a[kA])
        gA, gB = build(kA), build(kB)
        out = {}
        for key in gA:
            if key == "gphi" and gA["gphi"] is gA["gpsi"]:
                continue
            out[key] = (1.0 - t) * gA[key] + t * gB[key]
        if "gphi" not in out:
            out["gphi"] = out["gpsi"]
        return out
    return at


def initial_state(cfg, species_index, ids, grids0=None, sched=None):
    """Canonical initial state (x, q, q0, p) of the selected ids.

    Without pre-initial conditions q = q0 = p.  With them (cfg['pre_ic']),
    eq. transform is applied at a_i to the sampled p using the super-horizon
    moments delta = -2 psi and theta = k^2 tau psi / 2 (sec. 2.1), and the
    result is rounded once to binary32 like the sample itself.
    """
    sp = cfg["species"][species_index]
    L = cfg["box_mpc"]
    x = particles.positions_f64(sp["seed"], ids, L)
    p = particles.momenta_f64(sp["seed"], ids)
    q = p.copy()
    if cfg.get("pre_ic", False):
        a_i = sched["a"][0]
        d_grid, v_grid = grids0
        dlt = push.interpolate(d_grid, x, L)
        v = np.stack([push.interpolate(v_grid[d], x, L) for d in range(3)], axis=-1)
        q = particles.pre_initial_transform(p, dlt, v, sp["m"], a_i)
        q = q.astype(np.float32).astype(np.float64)
    return x, q, q.copy(), p


def super_horizon_grids(cfg, d0, a, tau):
    """delta = -2 psi and grad(nabla^-2 theta) with theta_k = k^2 tau psi_k / 2,
    evaluated from psi_k in Fourier space (sec. 2.1, initial conditions)."""
    G = cfg["grid_n"]
    L = cfg["box_mpc"]
    kx, ky, kz, kmag = field.wavevectors(G, L)
    safe = np.where(kmag > 0, kmag, 1.0)
    _, t_psi, _ = field.potential_transfers(safe, a, model_of(cfg))
    psi_k = np.where(kmag > 0, t_psi, 0.0) * d0
    delta_k = -2.0 * psi_k
    theta_k = 0.5 * kmag ** 2 * tau * psi_k
    inv_lap_theta = np.where(kmag > 0, -theta_k / safe ** 2, 0.0)

    def inv(fk):
        return sfft.irfftn(fk, s=(G, G, G), axes=(0, 1, 2), workers=os.cpu_count()) * float(G) ** 3
    d_grid = inv(delta_k)
    v_grid = np.stack([inv(1j * kv * inv_lap_theta) for kv in (kx, ky, kz)])
    return d_grid, v_grid


def run_particles(cfg, species_index, ids, k_end=None, d0=None, return_all=False):
    """Integrate the selected particle ids of one species; returns dict with
    x, q (final), q0, p and w (delta-f weights).  cfg['eom'] names the
    equations of motion (a key of push.EOM_BY_NAME; default 'separable') and
    cfg['interp_order'] the force interpolation (1 CIC, 2 TSC; default 1)."""
    sched = schedule(cfg)
    if d0 is None:
        d0 = delta0(cfg, cfg["species"][species_index]["field"])
    eom = cfg.get("eom", "separable")
    eom = push.EOM_BY_NAME[eom] if isinstance(eom, str) else int(eom)
    potentials = eom in (push.EOM_EXACT, push.EOM_CANONICAL)
    grids_at = grids_provider(cfg, d0, sched, with_psi=potentials, with_phi=potentials)
    pre = None
    if cfg.get("pre_ic", False):
        tau_i = background.conformal_time(sched["a"][0], *cosmo_args(cfg))
        pre = super_horizon_grids(cfg, d0, sched["a"][0], tau_i)
    x0, q, q0, p = initial_state(cfg, species_index, ids, pre, sched)
    m = cfg["species"][species_index]["m"]
    order = max(1, int(cfg.get("interp_order", 1)))
    if eom == push.EOM_SEPARABLE:
        x, q = push.kdk(x0, q, q0, m, sched, cfg["box_mpc"], grids_at, 0, k_end, order)
    else:
        x, q = push.kdk_variant(x0, q, m, sched, cfg["box_mpc"], grids_at, eom, 0, k_end, order)
    w = stats.deltaf_weights(q, p)
    out = dict(x=x, q=q, q0=q0, p=p, w=w, x0=x0, sched=sched)
    if return_all:
        out["d0"] = d0
    return out


def density_spectrum(cfg, species_index, res, mode="cross", a=None, analysis_n=0):
    """Binned P(k) of the energy-density contrast from an integrated full sample
    (res from run_particles over all ids).  mode 'cross' uses even and odd ids
    as the two halves; 'auto' uses all particles.  analysis_n: deposit mesh
    (default the configuration's G)."""
    G, L = analysis_n or cfg["grid_n"], cfg["box_mpc"]
    sp = cfg["species"][species_index]
    m = sp["m"]
    a = res["sched"]["a"][-1] if a is None else a
    eps = stats.energies(res["q"], m, a)
    mean_eps = background.mean_energy(m, a)
    n = res["x"].shape[0]
    ids = np.arange(n)
    if mode == "auto":
        d = stats.density_contrast(res["x"], res["w"], eps, G, L, n, mean_eps)
        return stats.binned_power(d, d, L, cfg["pk_bins"]), (d, d)
    halves = []
    for par in (0, 1):
        s = (ids % 2) == par
        halves.append(stats.density_contrast(res["x"][s], res["w"][s], eps[s], G, L,
                                             int(s.sum()), mean_eps))
    return stats.binned_power(halves[0], halves[1], L, cfg["pk_bins"]), tuple(halves)


def momentum_spectrum(cfg, species_index, res, mode="cross", a=None, analysis_n=0):
    """Binned P(k) of the momentum perturbation (1 + delta) theta (sec. 4)
    from an integrated full sample, halves and mesh as in density_spectrum."""
    G, L = analysis_n or cfg["grid_n"], cfg["box_mpc"]
    m = cfg["species"][species_index]["m"]
    a = res["sched"]["a"][-1] if a is None else a
    mean_eps = background.mean_energy(m, a)
    n = res["x"].shape[0]
    ids = np.arange(n)
    if mode == "auto":
        t = stats.momentum_divergence(res["x"], res["w"], res["q"], G, L, n, mean_eps)
        return stats.binned_power_fourier(t, t, L, cfg["pk_bins"])
    halves = []
    for par in (0, 1):
        s = (ids % 2) == par
        halves.append(stats.momentum_divergence(res["x"][s], res["w"][s], res["q"][s], G, L,
                                                int(s.sum()), mean_eps))
    return stats.binned_power_fourier(halves[0], halves[1], L, cfg["pk_bins"])


def total_density_spectrum(cfg, species_indices, results, mode="cross", a=None, analysis_n=0):
    """Binned P(k) of the total energy-density contrast of several species
    that share one field (sec. 2.2 eq. empirical_rho, per species, and the
    spectra of sec. 4).

    Each species s gives its own contrast delta_s of eq. empirical_rho
    (normalised by its own particle count and mean energy <eps>_s).  The
    relic species share one temperature (sec. 2), hence one number density,
    so their mean densities are proportional to <eps>_s(a) and the total is
        delta = sum_s <eps>_s delta_s / sum_s <eps>_s.
    Halves are the even and odd ids of every species (mode 'cross'); 'auto'
    uses all particles.  results[i] is run_particles over all ids of
    species_indices[i]."""
    G, L = analysis_n or cfg["grid_n"], cfg["box_mpc"]
    a = results[0]["sched"]["a"][-1] if a is None else a
    halves = [np.zeros((G, G, G)), np.zeros((G, G, G))]
    weights = []
    for si, res in zip(species_indices, results):
        m = cfg["species"][si]["m"]
        mean_eps = background.mean_energy(m, a)
        eps = stats.energies(res["q"], m, a)
        n = res["x"].shape[0]
        ids = np.arange(n)
        weights.append(mean_eps)
        if mode == "auto":
            d = stats.density_contrast(res["x"], res["w"], eps, G, L, n, mean_eps)
            halves[0] += mean_eps * d
            continue
        for par in (0, 1):
            s = (ids % 2) == par
            if s.any():
                halves[par] += mean_eps * stats.density_contrast(
                    res["x"][s], res["w"][s], eps[s], G, L, int(s.sum()), mean_eps)
    total = float(np.sum(weights))
    halves = [h / total for h in halves]
    if mode == "auto":
        return stats.binned_power(halves[0], halves[0], L, cfg["pk_bins"]), (halves[0], halves[0])
    return stats.binned_power(halves[0], halves[1], L, cfg["pk_bins"]), tuple(halves)
