"""CIC interpolation and the separable kick-drift-kick push (oracle side, sec. 3.3).

State: positions x (N, 3) in [0, L) Mpc, comoving momenta q (N, 3) eV, the
momenta q0 (N, 3) at the start of the integration, and the mass m [eV].
"""
import numpy as np


def cic_corners(x, G, L):
    """Cloud-in-cell corners and weights on the periodic mesh x_j = j L / G.

    u = x G / L, i = floor(u), t = u - i per axis; the 8 corners are
    (i + c) mod G for c in {0, 1}^3 with weight prod (1 - t) or t.
    Returns (idx (8, N, 3) int64, wts (8, N)).
    """
    u = np.asarray(x, dtype=np.float64) * (G / L)
    i = np.floor(u)
    t = u - i
    i = i.astype(np.int64)
    idx, wts = [], []
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                c = np.array([cx, cy, cz])
                idx.append((i + c) % G)
                wx = t[:, 0] if cx else 1.0 - t[:, 0]
                wy = t[:, 1] if cy else 1.0 - t[:, 1]
                wz = t[:, 2] if cz else 1.0 - t[:, 2]
                wts.append(wx * wy * wz)
    return np.stack(idx), np.stack(wts)


def tsc_points(x, G, L):
    """Triangular-shaped-cloud stencil (interpolation order r = 2, sec. 4).

    u = x G / L, nearest mesh point i = floor(u + 1/2), d = u - i in [-1/2, 1/2)
    per axis; the 27 points are (i + o) mod G for o in {-1, 0, 1}^3 with the
    product of the one-dimensional weights (1/2)(1/2 - d)^2, 3/4 - d^2 and
    (1/2)(1/2 + d)^2.  Returns (idx (27, N, 3) int64, wts (27, N)).
    """
    u = np.asarray(x, dtype=np.float64) * (G / L)
    i = np.floor(u + 0.5)
    d = u - i
    i = i.astype(np.int64)
    w1 = [0.5 * (0.5 - d) ** 2, 0.75 - d ** 2, 0.5 * (0.5 + d) ** 2]
    idx, wts = [], []
    for ox in range(3):
        for oy in range(3):
            for oz in range(3):
                o = np.array([ox, oy, oz]) - 1
                idx.append((i + o) % G)
                wts.append(w1[ox][:, 0] * w1[oy][:, 1] * w1[oz][:, 2])
    return np.stack(idx), np.stack(wts)


def interpolate(grid, x, L, order=1):
    """Value of a periodic (G, G, G) grid at positions x (N, 3): trilinear
    (CIC, order 1) or triangular-shaped cloud (TSC, order 2)."""
    G = grid.shape[0]
    idx, wts = cic_corners(x, G, L) if order == 1 else tsc_points(x, G, L)
    out = np.zeros(x.shape[0])
    for c in range(len(wts)):
        out += wts[c] * grid[idx[c, :, 0], idx[c, :, 1], idx[c, :, 2]]
    return out


def sample_fields(grids, x, L, order=1):
    """Gradients of psi and phi (N, 3) and phi-dot (N,) at the particles."""
    gpsi = np.stack([interpolate(grids["gpsi"][d], x, L, order) for d in range(3)], axis=-1)
    if grids["gphi"] is grids["gpsi"]:
        gphi = gpsi
    else:
        gphi = np.stack([interpolate(grids["gphi"][d], x, L, order) for d in range(3)], axis=-1)
    phidot = interpolate(grids["phidot"], x, L, order)
    return gpsi, gphi, phidot


def separable_force(q0, m, a, gpsi, gphi, phidot):
    """Right-hand side of eq. releq_approx (sec. 3.3):

    dq/dtau = -eps0 grad psi - (q0^2/eps0) grad phi + q0 (q0 . grad phi)/eps0 + q0 phidot,
    eps0 = sqrt(q0^2 + m^2 a^2), with q0 the momentum at the start.
    """
    q0sq = np.sum(q0 * q0, axis=-1)
    eps0 = np.sqrt(q0sq + (m * a) ** 2)
    q0_dot_gphi = np.sum(q0 * gphi, axis=-1)
    return (-eps0[:, None] * gpsi
            - (q0sq / eps0)[:, None] * gphi
            + q0 * (q0_dot_gphi / eps0)[:, None]
            + q0 * phidot[:, None])


def velocity(q, m, a):
    """Right-hand side of eq. geodesic_approx: dx/dtau = q / sqrt(q^2 + m^2 a^2)."""
    eps = np.sqrt(np.sum(q * q, axis=-1) + (m * a) ** 2)
    return q / eps[:, None]


def kdk(x, q, q0, m, sched, L, grids_at, k_begin=0, k_end=None, order=1):
    """Leapfrog of sec. 3.3 for steps k_begin .. k_end-1 of a schedule.

    Each step: q += dtau_k^{k+1/2} F(x_k, a_k); x += dtau_k^{k+1} v(q, a_{k+1/2})
    (mod L); q += dtau_{k+1/2}^{k+1} F(x_{k+1}, a_{k+1}).  The half-kicks are
    kept separate.  grids_at(k) returns the grid set at time a_k.  The drift
    uses a_{k+1/2}, the midpoint in log a.  order: force interpolation (1 CIC,
    2 TSC).  Returns new (x, q).
    """
    x = np.array(x, dtype=np.float64)
    q = np.array(q, dtype=np.float64)
    q0 = np.asarray(q0, dtype=np.float64)
    n = len(sched["drift"])
    k_end = n if k_end is None else k_end
    for k in range(k_begin, k_end):
        g = sample_fields(grids_at(k), x, L, order)
        q = q + sched["kick1"][k] * separable_force(q0, m, sched["a"][k], *g)
        x = x + sched["drift"][k] * velocity(q, m, sched["a_half"][k])
        x = np.mod(x, L)
        g = sample_fields(grids_at(k + 1), x, L, order)
        q = q + sched["kick2"][k] * separable_force(q0, m, sched["a"][k + 1], *g)
    return x, q


def reversed_schedule(sched):
    """The same time points traversed backward: a_k' = a_{n-k}, half-kicks and
    drift negated and reversed."""
    return dict(a=sched["a"][::-1].copy(), a_half=sched["a_half"][::-1].copy(),
                kick1=-sched["kick2"][::-1], kick2=-sched["kick1"][::-1],
                drift=-sched["drift"][::-1], tau_k=sched["tau_k"][::-1].copy(),
                delta_lna=-sched["delta_lna"])


# ---------------------------------------------------------------------------
# Other equations of motion (sec. 3.1, 3.2 and 5), integrated by an explicit
# kick-drift-kick that evaluates each half-kick with the momentum it starts
# from and the drift's metric factor at the start of the drift.  In the
# canonical form the momentum variable is P, sampled and weighted as if it
# were q (the substitution of P for q that sec. 4 compares against).
# ---------------------------------------------------------------------------
EOM_SEPARABLE, EOM_EXACT, EOM_CANONICAL, EOM_SR_NEWTON, EOM_SIMPLE_Q, EOM_NEWTONIAN = range(6)
EOM_BY_NAME = dict(separable=EOM_SEPARABLE, exact=EOM_EXACT, canonical=EOM_CANONICAL,
                   sr_newton=EOM_SR_NEWTON, simple_q=EOM_SIMPLE_Q, newtonian=EOM_NEWTONIAN)


def sample_potentials(grids, x, L, order=1):
    """gpsi, gphi (N, 3), phidot, psi, phi (N,) at the particles (absent -> 0)."""
    gpsi, gphi, phidot = sample_fields(grids, x, L, order)
    psi = interpolate(grids["psi"], x, L, order) if "psi" in grids else np.zeros(len(x))
    phi = interpolate(grids["phi"], x, L, order) if "phi" in grids else np.zeros(len(x))
    return gpsi, gphi, phidot, psi, phi


def variant_force(mode, q, m, a, gpsi, gphi, phidot):
    """Right-hand sides of the momentum equations:
      EXACT     eq. releq:      -eps grad psi - (q^2/eps) grad phi + q (q.grad phi)/eps + q phidot
      CANONICAL eq. releq_lag:  -eps grad psi - (P^2/eps) grad phi
      SR_NEWTON eq. p_eq:       -(2 P^2 + m^2 a^2) / sqrt(P^2 + m^2 a^2) grad psi
      SIMPLE_Q  eq. q_eq:       -sqrt(q^2 + m^2 a^2) grad psi
      NEWTONIAN (sec. 5):       -m a grad psi, the q -> 0 limit of eq. q_eq
    with eps = sqrt(q^2 + m^2 a^2) of the current momentum (q or P)."""
    q2 = np.sum(q * q, axis=-1)
    eps = np.sqrt(q2 + (m * a) ** 2)
    if mode == EOM_EXACT:
        qg = np.sum(q * gphi, axis=-1)
        return (-eps[:, None] * gpsi - (q2 / eps)[:, None] * gphi
                + q * (qg / eps)[:, None] + q * phidot[:, None])
    if mode == EOM_CANONICAL:
        return -eps[:, None] * gpsi - (q2 / eps)[:, None] * gphi
    if mode == EOM_SR_NEWTON:
        return -((2.0 * q2 + (m * a) ** 2) / eps)[:, None] * gpsi
    if mode == EOM_SIMPLE_Q:
        return -eps[:, None] * gpsi
    if mode == EOM_NEWTONIAN:
        return -(m * a) * gpsi
    raise ValueError(mode)


def variant_velocity(mode, q, m, a, psi, phi):
    """Right-hand sides of the position equations:
      EXACT     eq. geodesic:     (q/eps)(1 + phi + psi)
      CANONICAL eq. geodesic_lag: (P/eps)[1 + psi + (2 - P^2/eps^2) phi]
      SR_NEWTON, SIMPLE_Q, NEWTONIAN: q / sqrt(q^2 + m^2 a^2)."""
    q2 = np.sum(q * q, axis=-1)
    eps = np.sqrt(q2 + (m * a) ** 2)
    v = q / eps[:, None]
    if mode == EOM_EXACT:
        return v * (1.0 + phi + psi)[:, None]
    if mode == EOM_CANONICAL:
        return v * (1.0 + psi + (2.0 - q2 / eps ** 2) * phi)[:, None]
    return v


def kdk_variant(x, q, m, sched, L, grids_at, mode, k_begin=0, k_end=None, order=1):
    """Explicit leapfrog for the non-separable forms: for k = k_begin .. k_end-1
      q += dtau_k^{k+1/2} F(x_k, q, a_k);
      x += dtau_k^{k+1} v(q, a_{k+1/2}; phi, psi at x_k)   (mod L);
      q += dtau_{k+1/2}^{k+1} F(x_{k+1}, q, a_{k+1})."""
    x = np.array(x, dtype=np.float64)
    q = np.array(q, dtype=np.float64)
    n = len(sched["drift"])
    k_end = n if k_end is None else k_end
    for k in range(k_begin, k_end):
        gpsi, gphi, phidot, psi, phi = sample_potentials(grids_at(k), x, L, order)
        q = q + sched["kick1"][k] * variant_force(mode, q, m, sched["a"][k], gpsi, gphi, phidot)
        x = np.mod(x + sched["drift"][k] * variant_velocity(mode, q, m, sched["a_half"][k], psi, phi), L)
        gpsi, gphi, phidot, _, _ = sample_potentials(grids_at(k + 1), x, L, order)
        q = q + sched["kick2"][k] * variant_force(mode, q, m, sched["a"][k + 1], gpsi, gphi, phidot)
    return x, q


def geodesic_force_terms(q, m, a, gpsi, gphi, phidot):
    """The four contributions to dq/dtau of eq. releq (sec. 3.1, Fig. 2), each
    (N, 3): -eps grad psi, -(q^2/eps) grad phi, q (q . grad phi)/eps and
    q phidot, with eps = sqrt(q^2 + m^2 a^2) of the current momentum."""
    q2 = np.sum(q * q, axis=-1)
    eps = np.sqrt(q2 + (m * a) ** 2)
    qg = np.sum(q * gphi, axis=-1)
    return (-eps[:, None] * gpsi, -(q2 / eps)[:, None] * gphi,
            q * (qg / eps)[:, None], q * phidot[:, None])


def force_term_rms(grids, x, q, m, a, L, order=1):
    """Root mean square over particles of the magnitude of each term of
    geodesic_force_terms at positions x (4 values)."""
    gpsi, gphi, phidot = sample_fields(grids, x, L, order)
    terms = geodesic_force_terms(q, m, a, gpsi, gphi, phidot)
    return np.array([np.sqrt(np.mean(np.sum(t * t, axis=-1))) for t in terms])
