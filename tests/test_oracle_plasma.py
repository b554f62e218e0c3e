"""Pins of the oracle's plasma models.

- ADAF: the four-velocity is normalised (u.u = -1), the field is orthogonal to
  it (b.u = 0) with b.b = B^2; outside the ISCO in the equatorial plane the
  Keplerian velocity is a circular geodesic (zero radial acceleration);
  inside the ISCO the flow is the zero-angular-momentum observer (u_phi = 0).
- Snapshot: cell-centred trilinear interpolation is exact for fields linear
  in the grid coordinates, returns stored values at cell centres, clamps at
  the radial ends, is periodic in phi; u.u = -1 for arbitrary primitives.
"""
import numpy as np
import pytest

import oracle
from paper_2302_02733_amd import workloads as W

A = 0.9375
ADAF = W.ADAF


def _check_frame(a, r, th, p):
    g = oracle.metric(a, 1.0, r, th)
    u, b = p["u"], p["b"]
    assert u @ g @ u == pytest.approx(-1.0, abs=1e-13)
    assert abs(b @ g @ u) < 1e-13 * p["B"] * max(1.0, np.abs(u).max())
    assert b @ g @ b == pytest.approx(p["B"] ** 2, rel=1e-12)


def test_adaf_frame_invariants_at_random_points():
    rng = np.random.default_rng(3)
    for _ in range(200):
        r = 10 ** rng.uniform(np.log10(1.4), 3)
        th = rng.uniform(0.02, np.pi - 0.02)
        p = oracle.plasma(ADAF, A, 1.0, r, th, 0.3)
        assert p["valid"]
        _check_frame(A, r, th, p)


def test_adaf_profiles():
    n0, T0 = ADAF["n0_cgs"], ADAF["T0_K"]
    eq = oracle.plasma(ADAF, A, 1.0, 4.0, np.pi / 2, 0.0)
    assert eq["ne"] == pytest.approx(n0 / 8.0, rel=1e-14)
    assert eq["thetae"] == pytest.approx(1.380649e-16 * T0 / 4.0 / (9.1093837015e-28 * 2.99792458e10 ** 2), rel=1e-14)
    # one scale height above the plane (z = 0.5 r): factor exp(-1/2)
    r, th = 10.0, np.arccos(0.5)
    p = oracle.plasma(ADAF, A, 1.0, r, th, 0.0)
    assert p["ne"] == pytest.approx(n0 * r ** -1.5 * np.exp(-0.5), rel=1e-13)
    # beta = 10: B^2/(8 pi) = p_virial / beta, p_virial = n_e m_p c^2 / (6 r)
    pmag = p["B"] ** 2 / (8 * np.pi)
    assert pmag == pytest.approx(p["ne"] * 1.67262192369e-24 * 2.99792458e10 ** 2 / (6 * r) / 10.0, rel=1e-13)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9375])
def test_keplerian_flow_is_circular_geodesic_outside_isco(a):
    for r in (oracle.isco(a) + 0.01, 8.0, 30.0, 300.0):
        p = oracle.plasma(ADAF, a, 1.0, r, np.pi / 2, 0.0)
        G = oracle.christoffel(a, 1.0, r, np.pi / 2)
        u = p["u"]
        acc = np.einsum("mab,a,b->m", G, u, u)
        assert abs(acc[1]) < 1e-12 * (abs(u[0]) ** 2 / r ** 2)
        assert u[1] == 0 and u[2] == 0


def test_zamo_inside_isco():
    r = 0.5 * (oracle.horizon(A) + oracle.isco(A))
    p = oracle.plasma(ADAF, A, 1.0, r, 1.2, 0.0)
    g = oracle.metric(A, 1.0, r, 1.2)
    ul = g @ p["u"]
    assert abs(ul[3]) < 1e-13 * abs(ul[0])
    _check_frame(A, r, 1.2, p)


# ---------------- snapshot ----------------

SNAP = dict(n1=12, n2=10, n3=8, x1_start=np.log(1.2), dx1=(np.log(60.0) - np.log(1.2)) / 12,
            x2_start=0.0, dx2=0.1, x3_start=0.0, dx3=2 * np.pi / 8, hslope=0.3, gamma_ad=13 / 9,
            M_unit_g=1e19, R_high=40.0, R_low=1.0, sigma_cut=1e30, r_emit_max=1e30)
L_CM = 6.674e-8 * W.UNITS["M_bh_g"] / 2.99792458e10 ** 2
MP_ME = 1.67262192369e-24 + 9.1093837015e-28


def _centres(s):
    x1 = s["x1_start"] + (np.arange(s["n1"]) + 0.5) * s["dx1"]
    x2 = s["x2_start"] + (np.arange(s["n2"]) + 0.5) * s["dx2"]
    x3 = s["x3_start"] + (np.arange(s["n3"]) + 0.5) * s["dx3"]
    return x1, x2, x3


def _theta(x2, h):
    return np.pi * x2 + 0.5 * (1 - h) * np.sin(2 * np.pi * x2)


def _ne_to_rho(ne):
    rho_unit = SNAP["M_unit_g"] / L_CM ** 3
    return ne * MP_ME / rho_unit


def _make_prims(rho_fn, rng=None):
    x1, x2, x3 = _centres(SNAP)
    X1, X2, X3 = np.meshgrid(x1, x2, x3, indexing="ij")
    P = np.zeros((SNAP["n1"], SNAP["n2"], SNAP["n3"], 8))
    P[..., 0] = rho_fn(X1, X2, X3)
    P[..., 1] = 0.3
    if rng is not None:
        P[..., 2:5] = rng.normal(0, 0.3, P[..., 2:5].shape)
        P[..., 5:8] = rng.normal(0, 0.5, P[..., 5:8].shape)
    else:
        P[..., 7] = 0.1
    return P


def test_snapshot_trilinear_exact_for_linear_fields_and_centres():
    lin = lambda X1, X2, X3: 1.0 + 0.7 * X1 - 0.4 * X2
    P = _make_prims(lin)
    h = oracle.SnapshotHandle(SNAP, P)
    model = {"kind": oracle.MODEL_SNAPSHOT}
    rng = np.random.default_rng(5)
    x1c, x2c, x3c = _centres(SNAP)
    for _ in range(50):
        x1 = rng.uniform(x1c[0], x1c[-1])
        x2 = rng.uniform(x2c[0], x2c[-1])
        ph = rng.uniform(0, 2 * np.pi)
        r, th = np.exp(x1), _theta(x2, SNAP["hslope"])
        p = oracle.plasma(model, 0.5, 1.0, r, th, ph, L_CM, snap=h)
        assert _ne_to_rho(p["ne"]) == pytest.approx(lin(x1, x2, 0), rel=1e-12)
    # stored values at cell centres; clamped beyond the radial ends
    for (i, j, k) in [(0, 0, 0), (5, 4, 7), (11, 9, 3)]:
        r, th = np.exp(x1c[i]), _theta(x2c[j], SNAP["hslope"])
        p = oracle.plasma(model, 0.5, 1.0, r, th, x3c[k], L_CM, snap=h)
        assert _ne_to_rho(p["ne"]) == pytest.approx(P[i, j, k, 0], rel=1e-12)
    p_in = oracle.plasma(model, 0.5, 1.0, np.exp(x1c[0]) * 0.9, _theta(x2c[3], 0.3), 1.0, L_CM, snap=h)
    assert _ne_to_rho(p_in["ne"]) == pytest.approx(lin(x1c[0], x2c[3], 0), rel=1e-12)
    p_out = oracle.plasma(model, 0.5, 1.0, np.exp(x1c[-1]) * 1.5, _theta(x2c[3], 0.3), 1.0, L_CM, snap=h)
    assert _ne_to_rho(p_out["ne"]) == pytest.approx(lin(x1c[-1], x2c[3], 0), rel=1e-12)


def test_snapshot_periodic_in_phi():
    rng = np.random.default_rng(9)
    P = _make_prims(lambda X1, X2, X3: 1.0 + 0.0 * X1, rng)
    P[..., 0] = rng.uniform(0.5, 2.0, P[..., 0].shape)
    h = oracle.SnapshotHandle(SNAP, P)
    model = {"kind": oracle.MODEL_SNAPSHOT}
    for ph in (0.01, 3.0, 6.2):
        a = oracle.plasma(model, 0.5, 1.0, 7.0, 1.1, ph, L_CM, snap=h)
        b = oracle.plasma(model, 0.5, 1.0, 7.0, 1.1, ph + 2 * np.pi, L_CM, snap=h)
        c = oracle.plasma(model, 0.5, 1.0, 7.0, 1.1, ph - 4 * np.pi, L_CM, snap=h)
        assert a["ne"] == pytest.approx(b["ne"], rel=1e-12)
        assert a["ne"] == pytest.approx(c["ne"], rel=1e-12)


def test_snapshot_four_velocity_normalised_for_any_primitives():
    rng = np.random.default_rng(11)
    P = _make_prims(lambda X1, X2, X3: 1.0 + 0.0 * X1, rng)
    h = oracle.SnapshotHandle(SNAP, P)
    model = {"kind": oracle.MODEL_SNAPSHOT}
    a = 0.94
    for _ in range(40):
        r = np.exp(rng.uniform(np.log(1.5), np.log(50)))
        th = rng.uniform(0.1, np.pi - 0.1)
        p = oracle.plasma(model, a, 1.0, r, th, rng.uniform(0, 6.28), L_CM, snap=h)
        g = oracle.metric(a, 1.0, r, th)
        scale = np.abs(p["u"]) @ np.abs(g) @ np.abs(p["u"])
        assert p["u"] @ g @ p["u"] == pytest.approx(-1.0, abs=1e-14 * scale)
        assert abs(p["b"] @ g @ p["u"]) < 1e-12 * max(1.0, np.abs(p["b"]).max() * np.abs(p["u"]).max())
