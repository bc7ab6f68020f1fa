"""Seeded Gaussian field and linear metric potentials on the mesh (oracle side).

Discrete Fourier convention (the paper leaves it open; this is the reading used
throughout): for a mesh of G^3 points x_j = j L / G in a periodic box of side L,
    f(x_j) = sum_k f_k exp(i k.x_j),      f_k = G^-3 sum_j f(x_j) exp(-i k.x_j),
with k = (2 pi / L) n, n_a in [-G/2, G/2).  A Gaussian field with power
spectrum P(k) has <|delta_k|^2> = P(k) / V, V = L^3.

Half-complex storage: arrays of shape (G, G, G/2+1) hold the modes with
n_z >= 0; index (ix, iy, iz) is n = (ix or ix-G, iy or iy-G, iz).
"""
import os

import numpy as np
from scipy import fft as sfft, integrate

from . import philox
from .background import hubble, hubble0


# --------------------------------------------------------------------------
# Linear power spectrum (workload recipe: P(k) = A k^n_s T_BBKS^2, sigma_8)
# --------------------------------------------------------------------------

def bbks_transfer(k, gamma, h):
    """BBKS (Bardeen, Bond, Kaiser & Szalay 1986) transfer function.

    T(q) = ln(1 + 2.34 q) / (2.34 q) * [1 + 3.89 q + (16.1 q)^2 + (5.46 q)^3
           + (6.71 q)^4]^(-1/4),  q = k / (Gamma h)  with k in 1/Mpc.
    """
    k = np.asarray(k, dtype=np.float64)
    q = k / (gamma * h)
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.log1p(2.34 * q) / (2.34 * q) * poly ** -0.25
    return np.where(q > 0, t, 1.0)


def tophat_window(x):
    """Fourier transform of a real-space top-hat: 3 (sin x - x cos x) / x^3.

    Below x = 0.1 the Taylor series 1 - x^2/10 + x^4/280 - x^6/15120 + x^8/1330560
    replaces the closed form, which loses digits to cancellation there."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3
    x2 = x * x
    series = 1.0 - x2 / 10.0 + x2 ** 2 / 280.0 - x2 ** 3 / 15120.0 + x2 ** 4 / 1330560.0
    return np.where(np.abs(x) > 0.1, w, series)


def sigma_r_unnormalised(radius, ns, gamma, h):
    """sigma(R) for A = 1: sqrt( (2 pi^2)^-1 int k^2 k^ns T^2 W^2(kR) dk )."""
    def integrand(lnk):
        k = np.exp(lnk)
        return k ** 3 * k ** ns * bbks_transfer(k, gamma, h) ** 2 \
            * tophat_window(k * radius) ** 2
    # integrate in ln k; the integrand is negligible outside [1e-7, 1e3] / Mpc
    edges = np.linspace(np.log(1e-7), np.log(1e3), 41)
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(integrand, lo, hi, epsabs=1e-19, epsrel=1e-13, limit=400)
        total += val
    return np.sqrt(total / (2.0 * np.pi ** 2))


def power_amplitude(sigma8, ns, gamma, h):
    """A such that sigma(R = 8 Mpc/h) = sigma8 at z = 0 (D = 1)."""
    s = sigma_r_unnormalised(8.0 / h, ns, gamma, h)
    return (sigma8 / s) ** 2


def power_spectrum(k, amp, ns, gamma, h):
    """P(k) = A k^ns T_BBKS(k)^2  [Mpc^3]."""
    k = np.asarray(k, dtype=np.float64)
    return amp * k ** ns * bbks_transfer(k, gamma, h) ** 2


# --------------------------------------------------------------------------
# Mode geometry
# --------------------------------------------------------------------------

def mode_indices(G):
    """Integer wave numbers (nx, ny, nz) of the half-complex layout, broadcastable."""
    n = np.arange(G)
    n = np.where(n < G // 2, n, n - G)
    nx = n[:, None, None]
    ny = n[None, :, None]
    nz = np.arange(G // 2 + 1)[None, None, :]
    return nx, ny, nz


def wavevectors(G, L):
    """(kx, ky, kz, |k|) in 1/Mpc on the half-complex layout."""
    nx, ny, nz = mode_indices(G)
    kf = 2.0 * np.pi / L
    kx = kf * nx.astype(np.float64)
    ky = kf * ny.astype(np.float64)
    kz = kf * nz.astype(np.float64)
    kmag = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    return kx, ky, kz, kmag


def nyquist_or_zero_mask(G):
    """True where the mode is k = 0 or has any component at the Nyquist index G/2."""
    ix = np.arange(G)[:, None, None]
    iy = np.arange(G)[None, :, None]
    iz = np.arange(G // 2 + 1)[None, None, :]
    nyq = (ix == G // 2) | (iy == G // 2) | (iz == G // 2)
    zero = (ix == 0) & (iy == 0) & (iz == 0)
    return nyq | zero


# --------------------------------------------------------------------------
# Seeded Gaussian field delta_0(k) (linear density at z = 0)
# --------------------------------------------------------------------------

def gaussian_field(G, L, seed, amp, ns, gamma, h, fixed_amplitude=False):
    """delta_0(k) on the half-complex layout, complex128 (G, G, G/2+1).

    Each mode with linear index m = (ix G + iy)(G/2+1) + iz draws two uniforms
    u1, u2 from Philox(seed, field stream, m); the unit complex normal is
    z = sqrt(-ln u1) exp(2 pi i u2), so <|z|^2> = 1.  With fixed amplitudes
    (sec. 4: fixed initial conditions) |z| = 1.  delta_k = sqrt(P(k)/V) z.
    k = 0 and every mode with a Nyquist component are zero.  On the iz = 0
    plane, the mode with the larger linear index is set to the conjugate of
    its partner (-n_x, -n_y, 0), so the real-space field is real.
    """
    H = G // 2 + 1
    V = L ** 3
    _, _, _, kmag = wavevectors(G, L)
    pk = power_spectrum(np.where(kmag > 0, kmag, 1.0), amp, ns, gamma, h)
    delta = np.empty((G, G, H), dtype=np.complex128)

    def slab(ix):  # one slab at a time keeps memory modest; slabs are independent
        m = (ix * G + np.arange(G)[:, None]) * H + np.arange(H)[None, :]
        w = philox.draw(seed, philox.STREAM_FIELD, m)
        u1 = philox.to_unit_open(w[..., 0])
        u2 = philox.to_unit_open(w[..., 1])
        r = np.ones_like(u1) if fixed_amplitude else np.sqrt(-np.log(u1))
        phase = 2.0 * np.pi * u2
        delta[ix] = np.sqrt(pk[ix] / V) * r * (np.cos(phase) + 1j * np.sin(phase))

    if G >= 64:   # numpy releases the GIL in these array operations
        import concurrent.futures
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(slab, range(G)))
    else:
        for ix in range(G):
            slab(ix)
    delta[nyquist_or_zero_mask(G)] = 0.0
    # Hermitian symmetry on the iz = 0 plane
    plane = delta[:, :, 0]
    ix = np.arange(G)[:, None]
    iy = np.arange(G)[None, :]
    px = (G - ix) % G
    py = (G - iy) % G
    m_self = (ix * G + iy)
    m_partner = (px * G + py)
    take = m_self > m_partner
    partner_vals = np.conj(plane[px, py])
    delta[:, :, 0] = np.where(take, partner_vals, plane)
    return delta


# --------------------------------------------------------------------------
# Transfer functions of the potentials
# --------------------------------------------------------------------------

def radmat_growth(a, h, omega_m, omega_r):
    """Super-horizon potential in a radiation+matter universe, normalised to 1
    deep in matter domination, and its derivative d/da.

    With y = a / a_eq, a_eq = Omega_r / Omega_m and s = sqrt(1 + y), the
    Kodama-Sasaki solution Phi(y)/Phi(0) = (16 s + 9y^3 + 2y^2 - 8y - 16)/(10 y^3)
    is rewritten without cancellation as 1 - y (s^2 + 4s + 5) / (10 (s+1)^4);
    it falls from 1 to 9/10.  Returns (g, dg/da) with g = (10/9) Phi/Phi(0).
    This is a synthetic time-dependent model for exercising the phi-dot term and
    grid rebuilds; the paper's transfer functions come from a Boltzmann code.
    """
    a_eq = omega_r / omega_m
    y = np.asarray(a, dtype=np.float64) / a_eq
    s = np.sqrt(1.0 + y)
    num = y + 6.0 + 4.0 * s           # s^2 + 4 s + 5
    den = (s + 1.0) ** 4
    hfun = y * num / den
    dnum = 1.0 + 2.0 / s              # d(num)/dy
    dden = 4.0 * (s + 1.0) ** 3 / (2.0 * s)
    dh = (num + y * dnum) / den - y * num * dden / den ** 2
    g = (10.0 / 9.0) * (1.0 - hfun / 10.0)
    dg_dy = -(1.0 / 9.0) * dh
    return g, dg_dy / a_eq


def potential_transfers(kmag, a, model):
    """(T_phi, T_psi, T_phidot) at scale factor a for |k| > 0 (A1 reading).

    phi_k = T_phi delta_0(k), psi_k = T_psi delta_0(k), phidot_k = T_phidot delta_0(k)
    where phidot is the conformal-time derivative d phi / d tau = a^2 H d phi / d a.

    model keys: kind ('poisson' | 'radmat'), h, omega_m, omega_r, omega_l,
    slip_amp, slip_k.
      poisson: T_phi = -(3/2) H0^2 Omega_m D(a) / (a k^2) with D(a) = a (EdS),
               constant in time, so T_phidot = 0;
      radmat : the poisson form times the super-horizon factor g(a) above.
    psi = phi (1 - slip_amp exp(-k / slip_k)) (no slip when slip_amp = 0).
    """
    kmag = np.asarray(kmag, dtype=np.float64)
    h, om = model["h"], model["omega_m"]
    base = -1.5 * hubble0(h) ** 2 * om / kmag ** 2
    if model["kind"] == "poisson":
        t_phi = base
        t_phidot = np.zeros_like(base)
    elif model["kind"] == "radmat":
        g, dg = radmat_growth(a, h, om, model["omega_r"])
        hub = hubble(a, h, om, model["omega_r"], model.get("omega_l", 0.0))
        t_phi = base * g
        t_phidot = base * (a * a * hub * dg)
    else:
        raise ValueError("unknown potential model %r" % model["kind"])
    slip = 1.0 - model.get("slip_amp", 0.0) * np.exp(-kmag / model.get("slip_k", 1.0))
    return t_phi, t_phi * slip, t_phidot


def potential_grids(delta0, L, a, model, with_psi=False, with_phi=False):
    """Real-space gradient grids of psi and phi and the phi-dot grid (sec. 2.1).

    Returns dict with float64 arrays on the mesh x_j = j L / G:
      gpsi (3, G, G, G): d psi / d x_a,   gphi (3, G, G, G): d phi / d x_a,
      phidot (G, G, G), and psi / phi (G, G, G) when with_psi / with_phi.
    Gradients are spectral: d/dx_a -> i k_a.  The inverse transform is the
    unnormalised sum of the module docstring, i.e. G^3 * scipy.fft.irfftn.
    """
    G = delta0.shape[0]
    kx, ky, kz, kmag = wavevectors(G, L)
    safe_k = np.where(kmag > 0, kmag, 1.0)
    t_phi, t_psi, t_phidot = potential_transfers(safe_k, a, model)
    zero = kmag == 0
    t_phi = np.where(zero, 0.0, t_phi)
    t_psi = np.where(zero, 0.0, t_psi)
    t_phidot = np.where(zero, 0.0, t_phidot)

    def inv(fk):
        return sfft.irfftn(fk, s=(G, G, G), axes=(0, 1, 2), workers=os.cpu_count()) * float(G) ** 3

    psi_k = t_psi * delta0
    phi_k = t_phi * delta0
    out = {}
    out["gpsi"] = np.stack([inv(1j * kv * psi_k) for kv in (kx, ky, kz)])
    if np.array_equal(t_psi, t_phi):
        out["gphi"] = out["gpsi"]
    else:
        out["gphi"] = np.stack([inv(1j * kv * phi_k) for kv in (kx, ky, kz)])
    out["phidot"] = inv(t_phidot * delta0)
    if with_psi:
        out["psi"] = inv(psi_k)
    if with_phi:
        out["phi"] = inv(phi_k)
    return out
