"""Pins of the oracle's random numbers, background and schedule (CPU only)."""
import json
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import background, philox

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


# ---------------------------------------------------------------- Philox ----

@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (1, 0, 0, 0)),
    ((5, 7), (1, 0, 0, 0)),
    ((2 ** 64 - 1, 12345), (2 ** 40 + 3, 17, 2 ** 63, 9)),
    ((0xDEADBEEF, 0x46), (777, 3, 0, 0)),
])
def test_philox_matches_numpy_generator(key, ctr):
    """numpy.random.Philox implements the same published Philox4x64-10; its
    buffer is refilled after incrementing the counter, so starting from ctr-1
    its first four raw outputs are philox(ctr, key)."""
    start = np.array(ctr, dtype=np.uint64)
    start[0] -= np.uint64(1)  # ctr[0] >= 1 in the cases above
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
    ref = bg.random_raw(4)
    got = philox.philox4x64(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(got, ref)


def test_philox_vectorised_equals_scalar_calls():
    idx = np.array([1, 2, 3, 1000, 2 ** 33], dtype=np.uint64)
    many = philox.draw(99, philox.STREAM_POSITION, idx, trial=4)
    for i, v in enumerate(idx):
        one = philox.draw(99, philox.STREAM_POSITION, np.array([v]), trial=4)[0]
        assert np.array_equal(many[i], one)


def test_unit_interval_map_is_exact_and_open():
    w = np.array([0, 2 ** 64 - 1, 2 ** 63, 4096], dtype=np.uint64)
    u = philox.to_unit_open(w)
    assert u[0] == 2.0 ** -53 and u[1] == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))
    # exactness: (2j+1) 2^-53 recovers j
    j = (w >> np.uint64(12)).astype(np.float64)
    assert np.array_equal((u * 2.0 ** 53 - 1) / 2, j)


# ------------------------------------------------------------ background ----

def test_temperature_from_paper():
    assert GOLD["neutrino_temperature_K"]["value"] == background.T_NU_KELVIN
    assert background.t_nu_ev() == pytest.approx(1.680380e-4, rel=1e-6)


@pytest.mark.parametrize("z0,z1", [(1e9, 31.0), (1e6, 31.0), (1e9, 0.0), (5.0, 1e3)])
def test_eds_conformal_time_closed_form(z0, z1):
    """EdS: 1/(aH) = sqrt(a)/H0, so Delta tau = (2/H0)(sqrt(a1) - sqrt(a0))."""
    h = 0.7
    a0, a1 = 1 / (1 + z0), 1 / (1 + z1)
    got = background.dtau(np.log(a0), np.log(a1), h, 1.0)
    ref = 2.0 / background.hubble0(h) * (np.sqrt(a1) - np.sqrt(a0))
    assert got == pytest.approx(ref, rel=1e-13)


def test_radiation_matter_conformal_time_closed_form():
    """Omega_r + Omega_m: tau(a) = (2/(H0 Om)) (sqrt(Or + Om a) - sqrt(Or))."""
    h, om, orad = 0.7, 0.9999, 1e-4
    H0 = background.hubble0(h)
    for a in (1e-8, 1e-4, 1e-2, 1.0):
        ref = 2.0 / (H0 * om) * (np.sqrt(orad + om * a) - np.sqrt(orad))
        assert background.conformal_time(a, h, om, orad) == pytest.approx(ref, rel=1e-12)
    lo, hi = np.log(1e-6), np.log(3e-3)
    ref = 2.0 / (H0 * om) * (np.sqrt(orad + om * 3e-3) - np.sqrt(orad + om * 1e-6))
    assert background.dtau(lo, hi, h, om, orad) == pytest.approx(ref, rel=1e-12)


def test_schedule_structure():
    s = background.step_schedule(1e9, 0.0, 40, 0.7, 1.0)
    assert s["a"][0] == pytest.approx(1e-9, rel=1e-12) and s["a"][-1] == pytest.approx(1.0)
    ratios = s["a"][1:] / s["a"][:-1]
    assert np.allclose(ratios, ratios[0], rtol=1e-12)          # constant Delta log a
    assert np.allclose(s["a_half"], np.sqrt(s["a"][1:] * s["a"][:-1]), rtol=1e-12)
    assert np.allclose(s["kick1"] + s["kick2"], s["drift"], rtol=1e-12)
    assert np.all(s["kick1"] > 0) and np.all(s["kick2"] > s["kick1"])


def test_mean_energy_limits():
    """<eps> for m = 0 is <q> = 7 pi^4 T / (180 zeta(3)); for m a >> T,
    <eps> = m a (1 + <q^2>/(2 m^2 a^2) + O(a^-4)) with <q^2> = 15 zeta(5)/zeta(3) T^2."""
    T = background.t_nu_ev()
    q1 = float(7 * mp.pi ** 4 / (180 * mp.zeta(3)))
    q2 = float(15 * mp.zeta(5) / mp.zeta(3))
    assert q1 == pytest.approx(3.151374, abs=2e-6) and q2 == pytest.approx(12.93942, abs=2e-5)
    assert background.mean_energy(0.0, 1.0) == pytest.approx(q1 * T, rel=1e-12)
    ma = 1e4 * T
    e = background.mean_energy(1.0, ma)
    assert (e - ma) / ma == pytest.approx(q2 * T * T / (2 * ma * ma), rel=1e-6)
