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


def interpolate(grid, x, L):
    """Trilinear (CIC) value of a periodic (G, G, G) grid at positions x (N, 3)."""
    G = grid.shape[0]
    idx, wts = cic_corners(x, G, L)
    out = np.zeros(x.shape[0])
    for c in range(8):
        out += wts[c] * grid[idx[c, :, 0], idx[c, :, 1], idx[c, :, 2]]
    return out


def sample_fields(grids, x, L):
    """Gradients of psi and phi (N, 3) and phi-dot (N,) at the particles."""
    gpsi = np.stack([interpolate(grids["gpsi"][d], x, L) for d in range(3)], axis=-1)
    if grids["gphi"] is grids["gpsi"]:
        gphi = gpsi
    else:
        gphi = np.stack([interpolate(grids["gphi"][d], x, L) for d in range(3)], axis=-1)
    phidot = interpolate(grids["phidot"], x, L)
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


def kdk(x, q, q0, m, sched, L, grids_at, k_begin=0, k_end=None):
    """Leapfrog of sec. 3.3 for steps k_begin .. k_end-1 of a schedule.

    Each step: q += dtau_k^{k+1/2} F(x_k, a_k); x += dtau_k^{k+1} v(q, a_{k+1/2})
    (mod L); q += dtau_{k+1/2}^{k+1} F(x_{k+1}, a_{k+1}).  The half-kicks are
    kept separate.  grids_at(k) returns the grid set at time a_k.  The drift
    uses a_{k+1/2}, the midpoint in log a.  Returns new (x, q).
    """
    x = np.array(x, dtype=np.float64)
    q = np.array(q, dtype=np.float64)
    q0 = np.asarray(q0, dtype=np.float64)
    n = len(sched["drift"])
    k_end = n if k_end is None else k_end
    for k in range(k_begin, k_end):
        g = sample_fields(grids_at(k), x, L)
        q = q + sched["kick1"][k] * separable_force(q0, m, sched["a"][k], *g)
        x = x + sched["drift"][k] * velocity(q, m, sched["a_half"][k])
        x = np.mod(x, L)
        g = sample_fields(grids_at(k + 1), x, L)
        q = q + sched["kick2"][k] * separable_force(q0, m, sched["a"][k + 1], *g)
    return x, q


def reversed_schedule(sched):
    """The same time points traversed backward: a_k' = a_{n-k}, half-kicks and
    drift negated and reversed."""
    return dict(a=sched["a"][::-1].copy(), a_half=sched["a_half"][::-1].copy(),
                kick1=-sched["kick2"][::-1], kick2=-sched["kick1"][::-1],
                drift=-sched["drift"][::-1], tau_k=sched["tau_k"][::-1].copy(),
                delta_lna=-sched["delta_lna"])
