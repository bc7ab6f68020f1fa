"""Pins of the oracle's Gaussian field, spectral gradients and FFT conventions."""
import itertools

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import field

H, NS, GAMMA = 0.7, 0.965, 0.2


def test_bbks_limits():
    """T -> 1 for k -> 0; T ~ ln(2.34 q)/(2.34 q) (6.71 q)^-1 for q -> infinity."""
    assert field.bbks_transfer(1e-9, GAMMA, H) == pytest.approx(1.0, abs=1e-6)
    q = 1e6
    k = q * GAMMA * H
    asym = np.log(2.34 * q) / (2.34 * q) / (6.71 * q)
    assert field.bbks_transfer(k, GAMMA, H) == pytest.approx(asym, rel=1e-3)


def test_tophat_series_matches_closed_form_in_high_precision():
    mp.mp.dps = 50
    for x in (1e-5, 0.03, 0.0999, 0.1001, 2.0, 40.0):
        xm = mp.mpf(x)
        ref = 3 * (mp.sin(xm) - xm * mp.cos(xm)) / xm ** 3
        assert field.tophat_window(x) == pytest.approx(float(ref), rel=1e-13, abs=1e-17)


def test_sigma8_normalisation_independent_integrator():
    """sigma(8 Mpc/h) of the normalised spectrum is sigma_8, recomputed by a
    plain trapezoid rule in ln k on a dense grid (a different integrator)."""
    amp = field.power_amplitude(0.8, NS, GAMMA, H)
    lnk = np.linspace(np.log(1e-7), np.log(1e3), 2_000_001)
    k = np.exp(lnk)
    integrand = k ** 3 * field.power_spectrum(k, amp, NS, GAMMA, H) \
        * field.tophat_window(k * 8.0 / H) ** 2
    s2 = integrate.trapezoid(integrand, lnk) / (2 * np.pi ** 2)
    assert np.sqrt(s2) == pytest.approx(0.8, rel=1e-9)


def _full_from_half(half, G):
    """Complete a half-complex array to the full (G, G, G) spectrum by Hermitian symmetry."""
    full = np.zeros((G, G, G), dtype=complex)
    full[:, :, : G // 2 + 1] = half
    for ix, iy, iz in itertools.product(range(G), range(G), range(G // 2 + 1, G)):
        full[ix, iy, iz] = np.conj(half[(-ix) % G, (-iy) % G, (-iz) % G])
    return full


def test_field_is_hermitian_and_real():
    G, L = 8, 300.0
    amp = field.power_amplitude(0.8, NS, GAMMA, H)
    d = field.gaussian_field(G, L, 42, amp, NS, GAMMA, H)
    full = _full_from_half(d, G)
    # Hermitian symmetry holds on every plane, including the iz = 0 plane
    for ix, iy, iz in itertools.product(range(G), repeat=3):
        assert full[ix, iy, iz] == np.conj(full[(-ix) % G, (-iy) % G, (-iz) % G])
    real_space = np.fft.ifftn(full) * G ** 3
    assert np.max(np.abs(real_space.imag)) < 1e-12 * np.max(np.abs(real_space.real))
    # zeroed modes
    assert d[0, 0, 0] == 0
    assert np.all(d[G // 2] == 0) and np.all(d[:, G // 2] == 0) and np.all(d[:, :, G // 2] == 0)


def test_field_fixed_amplitude_exact():
    G, L = 16, 500.0
    amp = field.power_amplitude(0.8, NS, GAMMA, H)
    d = field.gaussian_field(G, L, 3, amp, NS, GAMMA, H, fixed_amplitude=True)
    _, _, _, k = field.wavevectors(G, L)
    mask = ~field.nyquist_or_zero_mask(G)
    ref = np.sqrt(field.power_spectrum(k[mask], amp, NS, GAMMA, H) / L ** 3)
    assert np.allclose(np.abs(d[mask]), ref, rtol=1e-14)


def test_field_power_statistics():
    """<|delta_k|^2> V / P(k) = 1 within sqrt(2 / N_modes) per shell, and the
    amplitude distribution |z|^2 is Exp(1) (mean 1, variance 1)."""
    G, L = 64, 800.0
    amp = field.power_amplitude(0.8, NS, GAMMA, H)
    d = field.gaussian_field(G, L, 11, amp, NS, GAMMA, H)
    _, _, _, k = field.wavevectors(G, L)
    mask = ~field.nyquist_or_zero_mask(G)
    ratio = (np.abs(d[mask]) ** 2 * L ** 3 / field.power_spectrum(k[mask], amp, NS, GAMMA, H))
    n = ratio.size
    assert abs(ratio.mean() - 1) < 5 / np.sqrt(n)
    assert abs(ratio.var() - 1) < 5 * np.sqrt(8 / n)
    # phases uniform: mean of exp(i theta) vanishes
    ph = np.angle(d[mask][k[mask] > 0])
    assert abs(np.mean(np.exp(1j * ph))) < 5 / np.sqrt(ph.size)


def test_single_mode_gradient_at_nodes():
    """A single Fourier mode delta_0 = c at n = (1, 2, 3): psi(x) = 2 Re(T c e^{ik.x}),
    so d psi/dx_a = -2 Im(k_a T c e^{ik.x}) exactly at the mesh points."""
    G, L = 16, 250.0
    model = dict(kind="poisson", h=H, omega_m=1.0, omega_r=0.0, slip_amp=0.0, slip_k=1.0)
    d = np.zeros((G, G, G // 2 + 1), dtype=complex)
    n = np.array([1, 2, 3])
    c = 0.3 - 0.7j
    d[n[0], n[1], n[2]] = c
    g = field.potential_grids(d, L, 1.0, model, with_psi=True)
    kv = 2 * np.pi / L * n
    T, _, _ = field.potential_transfers(np.linalg.norm(kv), 1.0, model)
    xs = np.arange(G) * L / G
    X = np.meshgrid(xs, xs, xs, indexing="ij")
    phase = np.exp(1j * (kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2]))
    psi_ref = 2 * np.real(T * c * phase)
    assert np.allclose(g["psi"], psi_ref, rtol=0, atol=1e-13 * np.abs(psi_ref).max())
    for a in range(3):
        ref = -2 * np.imag(kv[a] * T * c * phase)
        assert np.allclose(g["gpsi"][a], ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    assert np.all(g["phidot"] == 0)


def test_inverse_transform_matches_direct_dft():
    """Brute force on 4^3: sum_k f_k e^{ik.x_j} over the full spectrum."""
    G, L = 4, 100.0
    amp = field.power_amplitude(0.8, NS, GAMMA, H)
    d = field.gaussian_field(G, L, 5, amp, NS, GAMMA, H)
    model = dict(kind="poisson", h=H, omega_m=1.0, omega_r=0.0, slip_amp=0.0, slip_k=1.0)
    g = field.potential_grids(d, L, 1.0, model, with_psi=True)
    full = _full_from_half(d, G)
    nn = [i if i < G // 2 else i - G for i in range(G)]
    kf = 2 * np.pi / L
    ref = np.zeros((G, G, G))
    for jx, jy, jz in itertools.product(range(G), repeat=3):
        s = 0j
        for ix, iy, iz in itertools.product(range(G), repeat=3):
            kv = kf * np.array([nn[ix], nn[iy], nn[iz]])
            kk = np.linalg.norm(kv)
            if kk == 0:
                continue
            T, _, _ = field.potential_transfers(kk, 1.0, model)
            s += T * full[ix, iy, iz] * np.exp(2j * np.pi * (nn[ix] * jx + nn[iy] * jy + nn[iz] * jz) / G)
        ref[jx, jy, jz] = s.real
    assert np.allclose(g["psi"], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_slip_and_radmat_transfers():
    model = dict(kind="poisson", h=H, omega_m=1.0, omega_r=0.0, slip_amp=0.01, slip_k=1.0)
    k = np.array([1e-3, 0.1, 2.0])
    tphi, tpsi, tdot = field.potential_transfers(k, 0.3, model)
    H0 = 100 * H / 299792.458
    assert np.allclose(tphi, -1.5 * H0 ** 2 / k ** 2, rtol=1e-15)
    assert np.allclose(tpsi / tphi, 1 - 0.01 * np.exp(-k), rtol=1e-15)
    assert np.all(tdot == 0)
    # radiation + matter factor: limits 10/9 and 1, and the closed form of
    # Kodama & Sasaki evaluated in high precision
    g, _ = field.radmat_growth(np.array([1e-12, 1e6]), H, 1.0, 1e-4)
    assert g[0] == pytest.approx(10 / 9, rel=1e-7) and g[1] == pytest.approx(1.0, rel=1e-2)
    mp.mp.dps = 50
    for y in (0.01, 0.5, 3.0, 40.0):
        ym = mp.mpf(y)
        phi = (16 * mp.sqrt(1 + ym) + 9 * ym ** 3 + 2 * ym ** 2 - 8 * ym - 16) / (10 * ym ** 3)
        gg, dg = field.radmat_growth(y * 1e-4, H, 1.0, 1e-4)
        assert gg == pytest.approx(float(10 * phi / 9), rel=1e-13)
        d = mp.diff(lambda t: (10 / mp.mpf(9)) * (16 * mp.sqrt(1 + t) + 9 * t ** 3 + 2 * t ** 2 - 8 * t - 16)
                    / (10 * t ** 3), ym)
        assert dg == pytest.approx(float(d) / 1e-4, rel=1e-10)
