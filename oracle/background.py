"""Background cosmology and the time-step schedule (oracle side).

Units: lengths and conformal time in Mpc (c = 1), momenta/energies in eV,
H in 1/Mpc.
"""
import numpy as np
from scipy import integrate

C_KM_S = 299792.458            # speed of light [km/s]
K_B_EV_PER_K = 8.617333262e-5  # Boltzmann constant [eV/K]
T_NU_KELVIN = 1.95             # present neutrino temperature (sec. 2, below eq. def1)


def t_nu_ev():
    """k_B T with T = 1.95 K, in eV (sec. 2, below eq. def1)."""
    return T_NU_KELVIN * K_B_EV_PER_K


def hubble0(h):
    """H_0 = 100 h km/s/Mpc expressed in 1/Mpc."""
    return 100.0 * h / C_KM_S


def hubble(a, h, omega_m, omega_r=0.0, omega_l=0.0):
    """H(a) = H_0 sqrt(Omega_r a^-4 + Omega_m a^-3 + Omega_L)  [1/Mpc]."""
    a = np.asarray(a, dtype=np.float64)
    return hubble0(h) * np.sqrt(omega_r * a ** -4 + omega_m * a ** -3 + omega_l)


def dtau(lna0, lna1, h, omega_m, omega_r=0.0, omega_l=0.0):
    """Conformal time between two values of log a (sec. 3.3, step-size integral).

    Delta tau = int_{log a0}^{log a1} dlog a / (a H(a)), by adaptive quadrature.
    """
    def integrand(lna):
        a = np.exp(lna)
        return 1.0 / (a * hubble(a, h, omega_m, omega_r, omega_l))

    val, _ = integrate.quad(integrand, lna0, lna1, epsabs=0.0, epsrel=2e-14,
                            limit=200)
    return val


def step_schedule(z_begin, z_end, n_steps, h, omega_m, omega_r=0.0, omega_l=0.0):
    """Constant-Delta-log-a schedule of the leapfrog (sec. 3.3).

    Returns a dict of float64 arrays:
      a        (n+1,) scale factors a_k = a_i exp(k Delta)
      a_half   (n,)   a_{k+1/2} = a_i exp((k+1/2) Delta), the midpoint in log a
      tau_k    (n+1,) conformal time since the start, tau_k - tau_0
      kick1    (n,)   Delta tau_k^{k+1/2}   (opening half-kick of step k)
      kick2    (n,)   Delta tau_{k+1/2}^{k+1} (closing half-kick of step k)
      drift    (n,)   Delta tau_k^{k+1}
    A schedule with z_end > z_begin runs backward (negative Delta tau).
    """
    a_i = 1.0 / (1.0 + z_begin)
    a_f = 1.0 / (1.0 + z_end)
    lna_i = np.log(a_i)
    delta = (np.log(a_f) - lna_i) / n_steps
    lna = lna_i + delta * np.arange(n_steps + 1)
    lna_half = lna_i + delta * (np.arange(n_steps) + 0.5)
    cos = (h, omega_m, omega_r, omega_l)
    kick1 = np.array([dtau(lna[k], lna_half[k], *cos) for k in range(n_steps)])
    kick2 = np.array([dtau(lna_half[k], lna[k + 1], *cos) for k in range(n_steps)])
    drift = np.array([dtau(lna[k], lna[k + 1], *cos) for k in range(n_steps)])
    tau_k = np.concatenate([[0.0], np.cumsum(drift)])
    return dict(a=np.exp(lna), a_half=np.exp(lna_half), tau_k=tau_k,
                kick1=kick1, kick2=kick2, drift=drift, delta_lna=delta)


def conformal_time(a, h, omega_m, omega_r=0.0, omega_l=0.0):
    """tau(a) = int_0^a da' / (a'^2 H(a')), by quadrature (needs Omega_r or Omega_m > 0)."""
    def integrand(x):
        return 1.0 / (x * x * hubble(x, h, omega_m, omega_r, omega_l))
    val, _ = integrate.quad(integrand, 0.0, a, epsabs=0.0, epsrel=2e-14, limit=200)
    return val


def mean_energy(m_ev, a):
    """<eps>(a) = int q^2 sqrt(q^2 + m^2 a^2) fbar(q) dq / int q^2 fbar(q) dq  [eV].

    The Fermi-Dirac weighted mean energy per particle, the normalisation of the
    energy-density estimator of eq. empirical_rho (sec. 2.2, eq. rho_def).
    """
    T = t_nu_ev()
    ma = m_ev * a

    def num(x):  # x = q / T
        return x * x * np.sqrt((x * T) ** 2 + ma * ma) / (1.0 + np.exp(x))

    def den(x):
        return x * x / (1.0 + np.exp(x))

    n, _ = integrate.quad(num, 0.0, 200.0, epsabs=0.0, epsrel=2e-14, limit=400)
    d, _ = integrate.quad(den, 0.0, 200.0, epsabs=0.0, epsrel=2e-14, limit=400)
    return n / d
