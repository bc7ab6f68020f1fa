"""delta-f weights, energy-density deposit and binned power spectrum (oracle side)."""
import numpy as np

from .background import t_nu_ev
from .push import cic_corners


def fermi_dirac(q):
    """fbar(q) = 1 / (1 + exp(q / T)), T = 1.95 K (sec. 2, below eq. def1)."""
    return 1.0 / (1.0 + np.exp(np.asarray(q) / t_nu_ev()))


def deltaf_weights(q, p):
    """w = delta f / f = 1 - fbar(|q|) / fbar(|p|)  (sec. 2.2, weight definition).

    f at the particle is fbar(|p|) with p the initially sampled momentum
    (phase-space conservation) and delta f = fbar(|p|) - fbar(|q|).  Written
    without cancellation: with D = |q| - |p| = (2 p.d + d.d) / (|q| + |p|),
    d = q - p, the definition equals expm1(D/T) / (exp(-|p|/T) + exp(D/T)).
    """
    T = t_nu_ev()
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    d = q - p
    qn = np.sqrt(np.sum(q * q, axis=-1))
    pn = np.sqrt(np.sum(p * p, axis=-1))
    denom = qn + pn
    D = np.where(denom > 0,
                 (2.0 * np.sum(p * d, axis=-1) + np.sum(d * d, axis=-1)) / np.where(denom > 0, denom, 1.0),
                 0.0)
    return np.expm1(D / T) / (np.exp(-pn / T) + np.exp(D / T))


def energies(q, m, a):
    """eps = sqrt(q^2 + m^2 a^2) per particle."""
    return np.sqrt(np.sum(np.asarray(q) ** 2, axis=-1) + (m * a) ** 2)


def cic_deposit(x, values, G, L):
    """Sum of values * W_CIC onto the (G, G, G) mesh (adjoint of interpolation)."""
    idx, wts = cic_corners(x, G, L)
    grid = np.zeros((G, G, G))
    for c in range(8):
        np.add.at(grid, (idx[c, :, 0], idx[c, :, 1], idx[c, :, 2]), wts[c] * values)
    return grid


def density_contrast(x, w, eps, G, L, n_particles, mean_eps):
    """delta on the mesh from eq. empirical_rho (sec. 2.2).

    rho = rhobar + (M/N) sum_k w_k eps_k W(x - x_k) with the normalisation
    M/N = rhobar / (n <eps>), n = N / V, so that
    delta_j = G^3 / (N <eps>) sum_k w_k eps_k W_CIC(j, x_k).
    """
    return cic_deposit(x, w * eps, G, L) * (float(G) ** 3 / (n_particles * mean_eps))


def bin_index(n2, G, nbins):
    """Log bin of a mode with integer |n|^2 = n2 on [k_f, k_N), k = k_f sqrt(n2):
    b = floor(nbins * log(k/k_f) / log(k_N/k_f)) = floor(nbins log2(n2) / (2 log2(G/2))).
    Modes with n2 = 0 or b >= nbins are excluded (returned as -1)."""
    n2 = np.asarray(n2, dtype=np.float64)
    with np.errstate(divide="ignore"):
        b = np.floor(nbins * np.log2(np.where(n2 > 0, n2, 1.0)) / (2.0 * np.log2(G // 2)))
    b = b.astype(np.int64)
    return np.where((n2 > 0) & (b < nbins), b, -1)


def binned_power(delta_a, delta_b, L, nbins):
    """Power spectrum of two mesh fields in log bins (sec. 4).

    delta_k = G^-3 sum_j delta(x_j) exp(-i k.x_j) (numpy.fft.rfftn / G^3);
    Phat(k) = V Re(delta_a(k) conj(delta_b(k))): the cross spectrum of two
    halves of the sample, or the auto spectrum when delta_b is delta_a.
    Modes are counted over the full mesh: weight 1 on the n_z = 0 plane,
    2 elsewhere.  Returns (mean |k|, mean Phat, number of modes) per bin; an
    empty bin has NaN mean values.
    """
    G = delta_a.shape[0]
    fa = np.fft.rfftn(delta_a) / float(G) ** 3
    fb = fa if delta_b is delta_a else np.fft.rfftn(delta_b) / float(G) ** 3
    return binned_power_fourier(fa, fb, L, nbins)


def binned_power_fourier(fa, fb, L, nbins):
    """The binning of binned_power for two half-complex Fourier fields
    (G, G, G/2 + 1) already normalised as delta_k."""
    G = fa.shape[0]
    V = L ** 3
    p = V * np.real(fa * np.conj(fb))
    n = np.arange(G)
    n = np.where(n < G // 2, n, n - G)
    nz = np.arange(G // 2 + 1)
    n2 = n[:, None, None] ** 2 + n[None, :, None] ** 2 + nz[None, None, :] ** 2
    wgt = np.where(nz == 0, 1.0, 2.0)[None, None, :] * np.ones_like(p)
    kmag = (2.0 * np.pi / L) * np.sqrt(n2.astype(np.float64))
    b = bin_index(n2, G, nbins)
    sel = b >= 0
    cnt = np.bincount(b[sel], weights=wgt[sel], minlength=nbins)
    ksum = np.bincount(b[sel], weights=(wgt * kmag)[sel], minlength=nbins)
    psum = np.bincount(b[sel], weights=(wgt * p)[sel], minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        return ksum / cnt, psum / cnt, cnt


def momentum_divergence(x, w, q, G, L, n_particles, mean_eps):
    """Fourier field of the momentum perturbation (1 + delta) theta (sec. 4).

    The delta-f estimate of the energy-weighted velocity field,
      J(x_j) = G^3 / (N <eps>) sum_k w_k eps_k v_k W_CIC(j, x_k),  v = q / eps,
    i.e. the density contrast's deposit with w eps replaced by w q, so that
    (1 + delta) v = J; its divergence in Fourier space is
      Theta(k) = sum_a i k_a J_a(k)   (J_a(k) normalised as delta_k).
    Returns the half-complex (G, G, G/2 + 1) array."""
    from .field import wavevectors
    kx, ky, kz, _ = wavevectors(G, L)
    norm = float(G) ** 3 / (n_particles * mean_eps)
    theta = np.zeros((G, G, G // 2 + 1), dtype=np.complex128)
    for a, ka in enumerate((kx, ky, kz)):
        J = cic_deposit(x, w * q[:, a], G, L) * norm
        theta += 1j * ka * (np.fft.rfftn(J) / float(G) ** 3)
    return theta
