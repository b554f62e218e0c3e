"""Pins of the oracle's Kerr geometry against facts fixed outside the oracle.

- The Kerr-Schild metric equals the textbook Boyer-Lindquist Kerr metric under
  the coordinate change dt_BL = dt - 2r/Delta dr, dphi_BL = dphi - a/Delta dr.
- The metric is a vacuum solution: its Ricci tensor (from finite differences
  of the oracle's Christoffel symbols) vanishes.
- Analytic metric derivatives equal finite differences of the metric.
- The inverse metric multiplies to the identity; g^rr vanishes on the horizon.
- The ISCO radius minimises the circular-orbit energy.
"""
import numpy as np
import pytest

import oracle


def bl_metric(a, r, th):
    s2, c2 = np.sin(th) ** 2, np.cos(th) ** 2
    Sig = r * r + a * a * c2
    Delta = r * r - 2 * r + a * a
    g = np.zeros((4, 4))
    g[0, 0] = -(1 - 2 * r / Sig)
    g[0, 3] = g[3, 0] = -2 * a * r * s2 / Sig
    g[1, 1] = Sig / Delta
    g[2, 2] = Sig
    g[3, 3] = (r * r + a * a + 2 * a * a * r * s2 / Sig) * s2
    return g


POINTS = [(0.9375, 3.7, 1.1), (0.5, 12.0, 0.4), (-0.7, 2.9, 2.3), (0.0, 5.0, 1.5707963),
          (0.99, 2.5, 0.05)]


@pytest.mark.parametrize("a,r,th", POINTS)
def test_ks_equals_boyer_lindquist_transformed(a, r, th):
    Delta = r * r - 2 * r + a * a
    J = np.eye(4)
    J[0, 1] = -2 * r / Delta
    J[3, 1] = -a / Delta
    g_expect = J.T @ bl_metric(a, r, th) @ J
    g = oracle.metric(a, 1.0, r, th)
    np.testing.assert_allclose(g, g_expect, rtol=1e-12, atol=1e-12 * np.abs(g_expect).max())


@pytest.mark.parametrize("a,r,th", POINTS)
def test_inverse_metric_identity(a, r, th):
    g = oracle.metric(a, 1.0, r, th)
    gi = oracle.metric_inverse(a, 1.0, r, th)
    np.testing.assert_allclose(g @ gi, np.eye(4), atol=1e-13)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9375, 0.99])
def test_grr_vanishes_on_horizon(a):
    rh = oracle.horizon(a)
    assert abs(rh - (1 + np.sqrt(1 - a * a))) < 1e-15
    gi = oracle.metric_inverse(a, 1.0, rh, 1.0)
    assert abs(gi[1, 1]) < 1e-13


@pytest.mark.parametrize("a,r,th", POINTS)
@pytest.mark.parametrize("m", [0.0, 1.0])
def test_metric_derivatives_match_finite_differences(a, r, th, m):
    dg = oracle.metric_derivs(a, m, r, th)
    h = 1e-5
    for k, (dr, dt) in ((1, (h, 0)), (2, (0, h))):
        num = (oracle.metric(a, m, r + dr, th + dt) - oracle.metric(a, m, r - dr, th - dt)) / (2 * h)
        np.testing.assert_allclose(dg[k], num, atol=1e-8 * max(1.0, np.abs(num).max()))
    assert np.all(dg[0] == 0) and np.all(dg[3] == 0)


def christoffel_fd(a, m, r, th):
    g = oracle.metric(a, m, r, th)
    gi = np.linalg.inv(g)
    h = 1e-6
    dg = np.zeros((4, 4, 4))
    dg[1] = (oracle.metric(a, m, r + h, th) - oracle.metric(a, m, r - h, th)) / (2 * h)
    dg[2] = (oracle.metric(a, m, r, th + h) - oracle.metric(a, m, r, th - h)) / (2 * h)
    G = np.zeros((4, 4, 4))
    for mu in range(4):
        for al in range(4):
            for be in range(4):
                G[mu, al, be] = 0.5 * sum(gi[mu, nu] * (dg[al, nu, be] + dg[be, nu, al] - dg[nu, al, be])
                                          for nu in range(4))
    return G


@pytest.mark.parametrize("a,r,th", POINTS[:3])
def test_christoffel_from_numerical_metric(a, r, th):
    G = oracle.christoffel(a, 1.0, r, th)
    Gf = christoffel_fd(a, 1.0, r, th)
    np.testing.assert_allclose(G, Gf, atol=1e-7 * np.abs(Gf).max())


@pytest.mark.parametrize("a,r,th", [(0.9375, 3.7, 1.1), (0.5, 6.0, 0.7), (0.0, 4.0, 2.0)])
def test_kerr_is_ricci_flat(a, r, th):
    """R_mn = d_a G^a_mn - d_n G^a_ma + G^a_ab G^b_mn - G^a_nb G^b_ma = 0."""
    h = 1e-3
    G = oracle.christoffel(a, 1.0, r, th)

    def d(k):
        f = (lambda s: oracle.christoffel(a, 1.0, r + s, th)) if k == 1 else \
            (lambda s: oracle.christoffel(a, 1.0, r, th + s))
        return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)

    dG = np.zeros((4, 4, 4, 4))  # dG[k, mu, al, be] = d_k G^mu_al_be
    dG[1], dG[2] = d(1), d(2)
    R = (np.einsum("aamn->mn", dG) - np.einsum("nama->mn", dG)
         + np.einsum("aab,bmn->mn", G, G) - np.einsum("anb,bma->mn", G, G))
    scale = np.abs(np.einsum("aab,bmn->mn", G, G)).max() + np.abs(dG).max()
    assert np.abs(R).max() < 1e-8 * scale


def test_flat_mode_is_flat():
    """Mass factor 0 with a = 0: spherical coordinates of flat space."""
    r, th = 3.0, 0.8
    g = oracle.metric(0.0, 0.0, r, th)
    np.testing.assert_allclose(g, np.diag([-1, 1, r * r, (r * np.sin(th)) ** 2]), atol=1e-15)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9375, -0.5])
def test_isco_minimises_circular_orbit_energy(a):
    """Equatorial circular orbits: E(r) = -u_t with Omega = 1/(r^1.5 + a) has
    dE/dr = 0 at the ISCO (marginal stability)."""
    def energy(r):
        g = oracle.metric(a, 1.0, r, np.pi / 2)
        Om = 1.0 / (r ** 1.5 + a)
        ut = 1.0 / np.sqrt(-(g[0, 0] + 2 * g[0, 3] * Om + g[3, 3] * Om * Om))
        u = np.array([ut, 0, 0, Om * ut])
        return -(g @ u)[0]
    risco = oracle.isco(a)
    if a == 0.0:
        assert abs(risco - 6.0) < 1e-14
    h = 1e-4
    dE = (energy(risco + h) - energy(risco - h)) / (2 * h)
    assert abs(dE) < 1e-7
    assert energy(risco + 0.3) > energy(risco) and energy(risco - 0.1) > energy(risco)
