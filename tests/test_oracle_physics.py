"""Pins of the oracle's photon physics and detector response against
closed forms, conservation laws and independent quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O

ME = 510.99895
E0 = 159.0


@pytest.mark.parametrize("e", [30.0, 140.5, 159.0, 364.0, 1000.0])
@pytest.mark.parametrize("c", [-1.0, -0.3, 0.0, 0.7, 1.0])
def test_compton_energy_conserves_energy_and_momentum(e, c):
    # the recoil electron's kinetic energy T = E - E' and momentum p_e obey
    # T (T + 2 m c^2) = (p_e c)^2 = E^2 + E'^2 - 2 E E' cos(theta)
    ep = O.compton_energy(e, c)
    t = e - ep
    assert t * (t + 2 * ME) == pytest.approx(e * e + ep * ep - 2 * e * ep * c, rel=1e-12, abs=1e-9)


def test_compton_energy_monotone_and_forward_limit():
    cs = np.linspace(-1, 1, 101)
    ep = np.array([O.compton_energy(E0, c) for c in cs])
    assert np.all(np.diff(ep) > 0)
    assert ep[-1] == pytest.approx(E0, rel=1e-15)


@pytest.mark.parametrize("e", [20.0, 98.0, 121.27, 159.0, 511.0, 2000.0])
def test_kn_total_equals_integral_of_differential(e):
    # sigma / r_e^2 = 2 pi * int_{-1}^{1} (1/2) Psi(c) dc
    val, err = integrate.quad(lambda c: O.kn_shape(e, c), -1, 1, epsabs=1e-13, epsrel=1e-13)
    assert O.kn_total(e) == pytest.approx(math.pi * val, rel=1e-10)


def test_kn_thomson_and_high_energy_limits():
    # low-energy limit: sigma -> (8 pi / 3)(1 - 2k + O(k^2)), k = E / m c^2
    for k in (1e-2, 3e-3):
        ratio = O.kn_total(k * ME) / (8 * math.pi / 3)
        assert abs(ratio - (1 - 2 * k)) < 6 * k * k
    for c in (-1.0, 0.0, 0.5):
        assert O.kn_shape(1e-4, c) == pytest.approx(1 + c * c, rel=1e-5)
    k = 1e5
    asym = math.pi * (math.log(2 * k) + 0.5) / k
    assert O.kn_total(k * ME) == pytest.approx(asym, rel=2e-3)


def test_circle_mean_exact_for_periodic_rational():
    # int_0^{2 pi} dphi / (a - b cos phi) = 2 pi / sqrt(a^2 - b^2)
    k = E0 / ME
    a, b = 1 + k, k
    for m in (32, 64, 256):
        got = O.circle_mean(lambda p: 1.0 / (a - b * math.cos(p)), m)
        assert got == pytest.approx(1.0 / math.sqrt(a * a - b * b), rel=1e-13)


@pytest.mark.parametrize("e0", [80.0, 140.5, 159.0, 364.5])
def test_psi_bar_closed_form(e0):
    # with t = a - b cos(phi), a = 1 + k, b = k, Psi = t^-3 + t^-1 - sin^2 t^-2:
    # int t^-1 = 2 pi / r, int t^-3 = pi (2 a^2 + b^2) / r^5,
    # int sin^2 t^-2 = (a int t^-1 - 2 pi) / b^2, with r = sqrt(a^2 - b^2)
    k = e0 / ME
    a, b = 1 + k, k
    r = math.sqrt(a * a - b * b)
    j1 = 2 * math.pi / r
    j3 = math.pi * (2 * a * a + b * b) / r ** 5
    s2 = (a * j1 - 2 * math.pi) / (b * b)
    closed = (j3 + j1 - s2) / (2 * math.pi)
    assert O.psi_bar(e0, 512) == pytest.approx(closed, rel=1e-13)


def test_rho_is_ratio_of_integrated_cross_sections():
    def sig(e):
        return math.pi * integrate.quad(lambda c: O.kn_shape(e, c), -1, 1, epsabs=1e-13)[0]
    assert O.rho(E0, E0) == 1.0
    for e in (98.0, 110.0, 130.0, 150.0):
        assert O.rho(e, E0) == pytest.approx(sig(e) / sig(E0), rel=1e-9)
        assert O.rho(e, E0) > 1.0


@pytest.mark.parametrize("sigma", [0.17, 0.34])
def test_position_response(sigma):
    val = integrate.quad(lambda d: O.resp_K(d, sigma), -3 * sigma, 3 * sigma,
                         epsabs=1e-13, limit=200)[0]
    assert val == pytest.approx(1.0, rel=1e-10)
    assert O.resp_K(3 * sigma * (1 - 1e-9), sigma) == pytest.approx(0.0, abs=1e-8)
    assert O.resp_K(3 * sigma, sigma) == 0.0
    assert O.resp_K(0.3 * sigma, sigma) == O.resp_K(-0.3 * sigma, sigma)
    half = 5.0
    assert O.resp_D(0.0, half, sigma) == pytest.approx(1.0, rel=1e-13)
    assert O.resp_D(half, half, sigma) == pytest.approx(0.5, rel=1e-12)   # symmetric kernel
    assert O.resp_D(half + 3 * sigma, half, sigma) == pytest.approx(0.0, abs=1e-15)
    up = half - 0.7 * sigma
    ref = integrate.quad(lambda u: O.resp_K(u - up, sigma), -half, half, points=[up - 3 * sigma],
                         epsabs=1e-13, limit=200)[0]
    assert O.resp_D(up, half, sigma) == pytest.approx(ref, rel=1e-9)


def test_energy_response():
    s = 15.9 / (2 * math.sqrt(2 * math.log(2)))
    assert s == pytest.approx(6.752108312289752, rel=1e-14)
    val = integrate.quad(lambda e: O.resp_G(e, 130.0, s), 130.0 - 20 * s, 130.0 + 20 * s,
                         epsabs=1e-14)[0]
    assert val == pytest.approx(1.0, rel=1e-10)
    x = 11.3
    assert O.resp_W(E0, E0 - x, E0 + x, s) == pytest.approx(special.erf(x / (s * math.sqrt(2))),
                                                            rel=1e-13)
    for ep in (98.0, 121.3, 159.0):
        ref = integrate.quad(lambda e: O.resp_G(e, ep, s), 100.0, 175.0, epsabs=1e-14)[0]
        assert O.resp_W(ep, 100.0, 175.0, s) == pytest.approx(ref, rel=1e-10)
