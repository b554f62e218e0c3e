"""Pins of the oracle's thermal synchrotron coefficients.

- Bessel-function ratios agree with an independent library (SciPy), including
  the large-argument asymptotic branch.
- Frequency-integrated emissivity equals the total synchrotron power of a
  Maxwell-Juettner population (Larmor power 2 e^4 B^2 <gamma^2 beta^2>
  sin^2/(3 m^2 c^3), per steradian) to the accuracy of the fits.
- Frequency-integrated linear polarization is 75%, the single-electron value.
- Cold-plasma limit: rho_V and rho_Q equal the birefringence of the two
  magneto-ionic modes from the Appleton-Hartree refractive indices.
- Kirchhoff's law with the Planck function, realizability j_I >= |j_P|, and
  the parity of each coefficient under reversal of the field.
"""
import numpy as np
import pytest
from scipy import integrate, special

import oracle

C = 2.99792458e10
H = 6.62607015e-27
KB = 1.380649e-16
E = 4.803204712570263e-10
ME = 9.1093837015e-28


@pytest.mark.parametrize("x", [1e-3, 0.02, 0.5, 1.0, 3.7, 20.0, 150.0, 690.0])
def test_bessel_ratios_match_scipy(x):
    k0k2, k1k2 = oracle.bessel_ratios(x)
    assert k0k2 == pytest.approx(special.kve(0, x) / special.kve(2, x), rel=1e-13)
    assert k1k2 == pytest.approx(special.kve(1, x) / special.kve(2, x), rel=1e-13)


@pytest.mark.parametrize("x", [701.0, 900.0, 5e3, 1e6])
def test_bessel_ratio_asymptotic_branch(x):
    k0k2, k1k2 = oracle.bessel_ratios(x)
    assert k0k2 == pytest.approx(special.kve(0, x) / special.kve(2, x), rel=1e-14)
    assert k1k2 == pytest.approx(special.kve(1, x) / special.kve(2, x), rel=1e-14)


def _mean_gamma2beta2(theta):
    w = lambda g: g * np.sqrt(g * g - 1) * np.exp(-(g - 1) / theta)
    num = integrate.quad(lambda g: (g * g - 1) * w(g), 1, 1 + 80 * theta, limit=400)[0]
    den = integrate.quad(w, 1, 1 + 80 * theta, limit=400)[0]
    return num / den


def _integrated(theta, B, th, idx):
    ne = 1e5
    nuB = E * B / (2 * np.pi * ME * C)
    nuc = 1.5 * nuB * np.sin(th) * theta ** 2
    f = lambda lx: oracle.thermal_coefficients(ne, theta, B, nuc * 10 ** lx, np.cos(th))[idx] \
        * nuc * 10 ** lx * np.log(10)
    return integrate.quad(f, -8, 5, limit=400)[0], ne


@pytest.mark.parametrize("theta,th", [(50.0, 1.0), (100.0, 0.6)])
def test_total_power_matches_larmor(theta, th):
    B = 10.0
    jint, ne = _integrated(theta, B, th, 0)
    power = 2 * E ** 4 * B ** 2 * _mean_gamma2beta2(theta) * np.sin(th) ** 2 / (3 * ME ** 2 * C ** 3)
    expect = ne * power / (4 * np.pi)
    assert jint == pytest.approx(expect, rel=0.03)


def test_integrated_linear_polarization_is_three_quarters():
    jI, _ = _integrated(80.0, 10.0, 1.2, 0)
    jQ, _ = _integrated(80.0, 10.0, 1.2, 1)
    assert jQ / jI == pytest.approx(0.75, abs=0.015)


def _appleton_hartree_birefringence(ne, B, nu, th):
    X = ne * E * E / (np.pi * ME) / nu ** 2
    Y = E * B / (2 * np.pi * ME * C) / nu
    s2, c2 = np.sin(th) ** 2, np.cos(th) ** 2
    root = np.sqrt(0.25 * Y ** 4 * s2 * s2 + (1 - X) ** 2 * Y * Y * c2)
    n2 = [1 - X * (1 - X) / ((1 - X) - 0.5 * Y * Y * s2 + sgn * root) for sgn in (1, -1)]
    return 2 * np.pi * nu / C * abs(np.sqrt(n2[0]) - np.sqrt(n2[1]))


@pytest.mark.parametrize("th", [0.0, 0.3, 1.0, np.pi / 2, 2.5])
def test_cold_plasma_rotativities_match_appleton_hartree(th):
    ne, B, nu = 1e4, 30.0, 230e9
    c = oracle.thermal_coefficients(ne, 1e-7, B, nu, np.cos(th))
    rQ, rV = c[6], c[7]
    rho = np.hypot(rQ, rV)
    assert rho == pytest.approx(_appleton_hartree_birefringence(ne, B, nu, th), rel=1e-3)
    # the emissivities vanish for a cold plasma
    assert np.all(c[:6] == 0.0)
    # rotation measure form of rho_V: e^3 n B cos / (pi m^2 c^2 nu^2)
    assert rV == pytest.approx(E ** 3 * ne * B * np.cos(th) / (np.pi * ME ** 2 * C ** 2 * nu ** 2),
                               rel=1e-6, abs=1e-30)  # K0/K2 = 1 - O(theta_e)


@pytest.mark.parametrize("theta", [0.5, 3.0, 30.0])
def test_kirchhoff_with_planck_function(theta):
    nu = 230e9
    c = oracle.thermal_coefficients(3e5, theta, 20.0, nu, np.cos(0.8))
    T = theta * ME * C * C / KB
    Bnu = 2 * H * nu ** 3 / C ** 2 / np.expm1(H * nu / (KB * T))
    for k in range(3):
        assert c[3 + k] * Bnu == pytest.approx(c[k], rel=1e-13)
    assert c[0] > 0


def test_realizability_and_field_reversal():
    rng = np.random.default_rng(2)
    for _ in range(300):
        ne = 10 ** rng.uniform(2, 8)
        theta = 10 ** rng.uniform(-1, 2.5)
        B = 10 ** rng.uniform(-1, 3)
        nu = 10 ** rng.uniform(9, 13)
        cth = rng.uniform(-1, 1)
        c = oracle.thermal_coefficients(ne, theta, B, nu, cth)
        assert c[0] >= np.hypot(c[1], c[2]) * (1 - 1e-15)
        assert c[3] >= np.hypot(c[4], c[5]) * (1 - 1e-15)
        r = oracle.thermal_coefficients(ne, theta, B, nu, -cth)
        np.testing.assert_allclose(r[[0, 1, 3, 4, 6]], c[[0, 1, 3, 4, 6]], rtol=1e-14)
        np.testing.assert_allclose(r[[2, 5, 7]], -c[[2, 5, 7]], rtol=1e-14)


def test_no_plasma_gives_zero_coefficients():
    for args in [(0.0, 10.0, 5.0), (1e5, 0.0, 5.0), (1e5, 10.0, 0.0)]:
        assert np.all(oracle.thermal_coefficients(*args, 230e9, 0.3) == 0.0)


def test_field_along_ray_keeps_only_faraday_rotation():
    c = oracle.thermal_coefficients(1e5, 10.0, 20.0, 230e9, 1.0)
    assert np.all(c[:7] == 0.0) and c[7] > 0
