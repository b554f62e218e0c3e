"""Pins of the oracle's nonthermal (kappa) coefficient integrator.

Each test fixes a part of the integrator by something other than itself:
library Bessel functions, closed-form moments of the synchrotron functions,
their small- and large-argument limits, the thermal module's fits and
Bessel-function ratios in the thermal limit, Kirchhoff's law, the power-law
spectral indices and polarization degrees of Rybicki & Lightman (1979,
eqs. 6.36-6.38 and 6.53), and a brute-force scipy integration.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import gamma as G
from scipy.special import kv

import oracle

E = 4.803204712570263e-10
ME = 9.1093837015e-28
C = 2.99792458e10
KB = 1.380649e-16


def test_bessel_representations_match_library():
    x = np.array([1e-8, 1e-4, 0.03, 0.7, 3.0, 25.0, 300.0])
    for nu in (1 / 3, 2 / 3, 5 / 3):
        k, ki = oracle.bessel_k(nu, x)
        assert np.abs(k / kv(nu, x) - 1).max() < 1e-12
        for xi, kii in zip(x[2:6], ki[2:6]):
            ref = quad(lambda t: kv(nu, t), xi, np.inf, epsabs=0, epsrel=1e-13, limit=400)[0]
            assert abs(kii / ref - 1) < 1e-10


def test_synchrotron_function_moments():
    """int F = Gamma(2/3) Gamma(7/3), int G = Gamma(2/3) Gamma(4/3),
    int H = 2 Gamma(5/6) Gamma(7/6) (Mellin transform of K_nu)."""
    s = np.arange(np.log(1e-12), np.log(700.0), 0.02)
    X = np.exp(s)
    fgh = oracle.synchrotron_kernels(X)
    mom = (fgh * X[:, None]).sum(0) * 0.02
    ref = np.array([G(2 / 3) * G(7 / 3), G(2 / 3) * G(4 / 3), 2 * G(5 / 6) * G(7 / 6)])
    assert np.abs(mom / ref - 1).max() < 1e-9


def test_synchrotron_function_limits_and_identity():
    X = np.array([1e-9, 1e-7])
    F, Gf, H = oracle.synchrotron_kernels(X).T
    # R&L 6.34a and the small-argument form of K_{2/3}: F -> 4 pi/(sqrt3 Gamma(1/3)) (X/2)^(1/3), G/F -> 1/2
    lim = 4 * math.pi / (math.sqrt(3) * G(1 / 3)) * (X / 2) ** (1 / 3)
    assert np.abs(F / lim - 1).max() < 2e-5
    assert np.abs(Gf / F - 0.5).max() < 2e-5
    # H -> int_0^inf K_{1/3} = pi / sqrt(3)
    assert np.abs(H / (math.pi / math.sqrt(3)) - 1).max() < 1e-4
    # large X: F, G -> sqrt(pi X / 2) e^-X
    X = np.array([200.0, 400.0])
    F, Gf, H = oracle.synchrotron_kernels(X).T
    asy = np.sqrt(np.pi * X / 2) * np.exp(-X)
    assert np.abs(F / asy - 1).max() < 5e-3 and np.abs(Gf / asy - 1).max() < 5e-3
    # recurrence: int_X^inf K_{5/3} = 2 K_{2/3}(X) - int_X^inf K_{1/3}
    X = np.array([0.01, 0.5, 4.0])
    F = oracle.synchrotron_kernels(X)[:, 0]
    k23, _ = oracle.bessel_k(2 / 3, X)
    _, ki13 = oracle.bessel_k(1 / 3, X)
    assert np.abs(F / (X * (2 * k23 - ki13)) - 1).max() < 1e-12


def _thermal_pair(w, X, cth=0.5, ne=1e6, B=10.0):
    nuB = E * B / (2 * math.pi * ME * C)
    s = math.sqrt(1 - cth * cth)
    nu = X * 1.5 * nuB * s * w * w
    th = oracle.thermal_coefficients(ne, w, B, nu, cth)
    mj = oracle.kappa_coefficients(0.0, ne, w, B, nu, cth, dist=oracle.DIST_THERMAL)
    return th, mj, nu


@pytest.mark.parametrize("w", [10.0, 30.0, 100.0])
def test_thermal_limit_matches_thermal_module(w):
    """A Maxwell-Juttner input gives the thermal fits' emissivities within the
    fits' accuracy (Dexter's fits: about 1%), the Faraday rotativity exactly
    (K0/K2) and the conversion rotativity (K1/K2 + 6 Theta) at high X."""
    for X in (0.1, 1.0, 10.0, 100.0, 1000.0):
        th, mj, nu = _thermal_pair(w, X)
        for k in range(3):
            assert abs(mj[k] / th[k] - 1) < 0.02, (k, X, mj[k] / th[k])
        assert abs(mj[7] / th[7] - 1) < 1e-10
    th, mj, nu = _thermal_pair(w, 1e9)
    assert abs(mj[6] / th[6] - 1) < 1e-6


def test_kirchhoff_for_thermal_distribution():
    """alpha_S B_nu = j_S for a Maxwell-Juttner distribution (Rayleigh-Jeans
    B_nu; the Planck form differs by h nu / k T ~ 1e-9 here)."""
    for w, X in ((3.0, 2.0), (50.0, 300.0)):
        th, mj, nu = _thermal_pair(w, X)
        brj = 2 * nu * nu * w * ME
        for k in range(3):
            assert abs(mj[3 + k] * brj / mj[k] - 1) < 1e-12
            assert abs(mj[3 + k] / th[3 + k] - mj[k] / th[k]) < 1e-8


def test_large_kappa_tends_to_thermal():
    inp = np.array([[2e4, 5.0, 30.0], [2e4, 40.0, 3.0]])
    k = oracle.kappa_integrals(inp)
    t = oracle.kappa_integrals(inp, dist=oracle.DIST_THERMAL)
    assert np.abs(k / t - 1).max() < 3e-3


@pytest.mark.parametrize("kap", [3.5, 5.0, 7.0])
def test_power_law_tail(kap):
    """Far above the peak the kappa tail is a power law with p = kappa - 1:
    j ~ nu^-(p-1)/2 (I_F ~ X^-(kappa-2)/2), alpha ~ nu^-(p+4)/2 (A_F ~
    X^-(kappa-1)/2), linear polarization (p+1)/(p+7/3) in emission and
    (p+2)/(p+10/3) in absorption."""
    X1, X2 = 1e6, 2e6
    o = oracle.kappa_integrals(np.array([[kap, 1.0, X1], [kap, 1.0, X2]]))
    sl = np.log(o[1] / o[0]) / np.log(X2 / X1)
    p = kap - 1
    assert abs(sl[0] + (p - 1) / 2) < 0.02 * (p - 1) / 2 + 0.01
    assert abs(sl[3] + p / 2) < 0.02 * p / 2 + 0.01
    assert abs(o[0, 1] / o[0, 0] - (p + 1) / (p + 7 / 3)) < 0.01
    assert abs(o[0, 4] / o[0, 3] - (p + 2) / (p + 10 / 3)) < 0.01


def _brute(kap, w, X):
    """Adaptive scipy quadrature over the Lorentz factor of the integrands,
    written out from their definitions (the synchrotron functions, pinned
    above, from the oracle)."""
    def kern(Xg):
        return oracle.synchrotron_kernels(np.array([Xg]))[0]

    def shape(gm1):
        g = 1 + gm1
        return g * math.sqrt(gm1 * (g + 1)) * (1 + gm1 / (kap * w)) ** (-(kap + 1))

    def integ(fn):
        return quad(lambda v: fn(math.exp(v)) * math.exp(v), -40, 40, epsabs=0, epsrel=1e-10,
                    limit=800)[0]

    def xg(gm1):
        return X * w * w / (1 + gm1) ** 2

    norm = integ(shape)
    out = [integ(lambda q: shape(q) * kern(xg(q))[0]),
           integ(lambda q: shape(q) * kern(xg(q))[1]),
           integ(lambda q: shape(q) * kern(xg(q))[2] / (1 + q)),
           integ(lambda q: shape(q) * (kap + 1) / (kap * w + q) * kern(xg(q))[0]),
           integ(lambda q: shape(q) * (2 * (1 + q) - 1 / (1 + q)) * xg(q) / (1 + xg(q))),
           integ(lambda q: shape(q) * math.acosh(1 + q) / ((1 + q) * math.sqrt(q * (q + 2))))]
    return np.array(out) / norm


@pytest.mark.parametrize("kap,w,X", [(4.0, 3.0, 20.0), (7.5, 60.0, 0.05), (3.1, 1.5, 3e4)])
def test_integrator_against_brute_force(kap, w, X):
    o = oracle.kappa_integrals(np.array([[kap, w, X]]))[0]
    b = _brute(kap, w, X)
    got = o[[0, 1, 2, 3, 6, 7]]
    assert np.abs(got / b - 1).max() < 1e-8, got / b


def test_physical_guards():
    z = oracle.kappa_coefficients(5.0, 0.0, 10.0, 10.0, 230e9, 0.3)
    assert np.all(z == 0.0)
    along = oracle.kappa_coefficients(5.0, 1e6, 10.0, 10.0, 230e9, 1.0)
    assert np.all(along[:7] == 0.0) and along[7] > 0.0
    c = oracle.kappa_coefficients(5.0, 1e6, 10.0, 10.0, 230e9, 0.3)
    assert np.all(c > 0.0)
    assert math.hypot(c[1], c[2]) <= c[0] and math.hypot(c[4], c[5]) <= c[3]
    cm = oracle.kappa_coefficients(5.0, 1e6, 10.0, 10.0, 230e9, -0.3)
    assert np.allclose(cm[[0, 1, 3, 4, 6]], c[[0, 1, 3, 4, 6]], rtol=1e-14)
    assert np.allclose(cm[[2, 5, 7]], -c[[2, 5, 7]], rtol=1e-14)


@pytest.mark.parametrize("kap", [4.0, 6.0])
def test_rotativities_cold_limit(kap):
    """A cold kappa plasma (width w -> 0) rotates and converts like a cold
    electron gas: rho_V -> 2 n e^2 nu_B cos(theta) / (m c nu^2) (the
    textbook Faraday rotation rate, twice the rotation-measure rate
    e^3 n B cos(theta) / (2 pi m^2 c^2 nu^2)) and rho_Q -> n e^2 nu_B^2
    sin^2(theta) / (m c nu^3) (the quadratic birefringence of the
    Appleton-Hartree indices).  This fixes both rotativity weights at
    g -> 1 independently of the thermal module; between the cold and the
    thermal high-frequency limits the kappa weights are a reading."""
    ne, B, nu = 1e6, 10.0, 230e9
    nuB = E * B / (2 * math.pi * ME * C)
    for cth in (0.3, -0.8):
        s2 = 1 - cth * cth
        c = oracle.kappa_coefficients(kap, ne, 1e-5, B, nu, cth)
        rv = 2 * ne * E * E * nuB * cth / (ME * C * nu * nu)
        rq = ne * E * E * nuB * nuB * s2 / (ME * C * nu ** 3)
        assert abs(c[7] / rv - 1) < 1e-3, c[7] / rv
        assert abs(c[6] / rq - 1) < 1e-3, c[6] / rq
