"""Initial particle sample (oracle side).

Positions are uniform in the periodic box and momenta are drawn from the
homogeneous Fermi-Dirac distribution (sec. 2.1, sampling paragraph).  The
canonical initial state is the one both the FP64 and the FP32 forms start
from: positions on the 2^-32 L lattice (x = L u / 2^32 with u a uint32) and
momentum components rounded once to binary32.
"""
import numpy as np

from . import philox
from .background import t_nu_ev

MAX_TRIALS = 64


def positions_u32(seed, ids):
    """uint32 (N, 3): the high 32 bits of Philox(seed, position stream, id) words 0-2."""
    w = philox.draw(seed, philox.STREAM_POSITION, np.asarray(ids, dtype=np.uint64))
    return (w[..., :3] >> np.uint64(32)).astype(np.uint32)


def positions_f64(seed, ids, L):
    """Canonical positions in [0, L): x = L u / 2^32 (exact in binary64)."""
    return positions_u32(seed, ids).astype(np.float64) * (L / 2.0 ** 32)


def momentum_magnitude(seed, ids):
    """|q| [eV] with pdf proportional to q^2 fbar(q), fbar = 1 / (1 + exp(q/T)).

    Rejection from a Gamma(3, T) proposal q = -T ln(u1 u2 u3), which has pdf
    proportional to q^2 exp(-q/T); the ratio of target to proposal is
    1 / (1 + exp(-q/T)) <= 1, so a proposal is kept when
    u4 (1 + exp(-q/T)) < 1.  Trial t uses Philox(seed, momentum stream, id, t);
    the first kept trial wins (after MAX_TRIALS the last proposal is used,
    probability ~1e-65).
    """
    ids = np.asarray(ids, dtype=np.uint64)
    T = t_nu_ev()
    q = np.full(ids.shape, np.nan)
    done = np.zeros(ids.shape, dtype=bool)
    for trial in range(MAX_TRIALS):
        w = philox.draw(seed, philox.STREAM_MOMENTUM, ids, trial)
        u = philox.to_unit_open(w)
        prop = -T * np.log(u[..., 0] * u[..., 1] * u[..., 2])
        keep = (u[..., 3] * (1.0 + np.exp(-prop / T)) < 1.0) | (trial == MAX_TRIALS - 1)
        take = keep & ~done
        q[take] = prop[take]
        done |= keep
        if done.all():
            break
    return q


def directions(seed, ids):
    """Isotropic unit vectors: mu = 2 u1 - 1, phi = 2 pi u2."""
    w = philox.draw(seed, philox.STREAM_DIRECTION, np.asarray(ids, dtype=np.uint64))
    u = philox.to_unit_open(w)
    mu = 2.0 * u[..., 0] - 1.0
    ph = 2.0 * np.pi * u[..., 1]
    st = np.sqrt(1.0 - mu * mu)
    return np.stack([st * np.cos(ph), st * np.sin(ph), mu], axis=-1)


def momenta_f64(seed, ids):
    """Canonical momenta (N, 3) [eV]: |q| n_hat in binary64, rounded once to binary32."""
    q = momentum_magnitude(seed, ids)[..., None] * directions(seed, ids)
    return q.astype(np.float32).astype(np.float64)


def pre_initial_transform(q, delta, grad_inv_lap_theta, m_ev, a):
    """Pre-initial conditions, eq. transform (sec. 2.1).

    q_i -> q_i [1 + delta/nu + omega eps / (nu q_i) d_i(nabla^-2 theta)],
    with nu = 4, omega = 4/3 and eps = sqrt(q^2 + m^2 a^2) of the unperturbed
    sample.  delta (N,) and grad_inv_lap_theta (N, 3) are the super-horizon
    moments interpolated at the particles.  The bracket is multiplied out so
    that a vanishing component q_i needs no division.
    """
    nu = 4.0
    omega = 4.0 / 3.0
    eps = np.sqrt(np.sum(q * q, axis=-1) + (m_ev * a) ** 2)
    return q * (1.0 + delta[..., None] / nu) + (omega * eps / nu)[..., None] * grad_inv_lap_theta
