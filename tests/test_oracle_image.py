"""Whole-image pin of the oracle (the paper's images are not available):
convergence in eps.  The transfer is second order (Strang splitting, Heun
transport) on fourth-order geodesics, so the total flux approaches its limit
with differences shrinking about fourfold per halving of eps.

(No reflection symmetry is exact for these models: the ADAF rotates, and its
toroidal field, a pseudovector, keeps its sense across the equator, so the
mirror image of the plasma has the opposite field below the plane; Faraday
rotation and circular terms are odd in the field and feed back on I.)
"""
import numpy as np

import oracle
from paper_2302_02733_amd import workloads as W


def test_total_flux_converges_in_eps():
    fl = []
    for eps in (0.04, 0.02, 0.01):
        cam = W.adaf_camera(8, eps=eps, fov=30.0)
        S, st, ns = oracle.render(cam, W.UNITS, W.ADAF)
        fl.append(oracle.reduce(cam, W.UNITS, S)[0][0])
    d1, d2 = fl[0] - fl[1], fl[1] - fl[2]
    ratio = d1 / d2
    assert abs(d2) / fl[2] < 1e-2
    assert 2.0 < ratio < 8.0, (fl, ratio)


def test_parity_images_are_realizable():
    """P12 on the oracle's own parity images (the 64^2 ADAF and the 48^2
    snapshot, the images the GPU is compared with in full): I >= 0 and
    I^2 (1 + 1e-12) >= Q^2 + U^2 + V^2 at every pixel."""
    for name in ("adaf64", "snap48"):
        w = W.workload(name)
        snap = None
        if "snapshot" in w:
            desc, seed = w["snapshot"]
            snap = oracle.SnapshotHandle(desc, W.make_snapshot(desc, seed))
        S, st, ns = oracle.render(w["camera"], w["units"], w["model"], snap=snap)
        I, Q, U, V = S
        assert np.all(I >= 0) and I.max() > 0
        assert np.all(I * I * (1 + 1e-12) >= Q * Q + U * U + V * V), name


def test_empty_point_reading_is_within_the_truncation_error():
    """Both sides leave N unchanged at points where every coefficient is
    zero (no plasma), instead of projecting it on the fluid legs and
    rebuilding it there as the update is first stated.  The two readings
    differ only through the Heun transport of the components along K that
    the rebuild would drop, so the difference is a truncation error of the
    second-order transfer: on the 48^2 snapshot image it falls fourfold per
    halving of eps, and at the parity step (eps = 0.01) it is below 1e-6 of
    the total flux."""
    w = W.workload("snap48")
    desc, seed = w["snapshot"]
    snap = oracle.SnapshotHandle(desc, W.make_snapshot(desc, seed))
    diff = []
    for eps in (0.02, 0.01):
        cam = dict(w["camera"], eps=eps)
        S0, st0, ns0 = oracle.render(cam, w["units"], w["model"], snap=snap)
        S1, st1, ns1 = oracle.render(cam, w["units"], dict(w["model"], update_empty=1), snap=snap)
        assert np.array_equal(st0, st1) and np.array_equal(ns0, ns1)
        f0 = S0[0].sum()
        diff.append(max(abs(S1[k].sum() - S0[k].sum()) / f0 for k in range(4)))
    assert 0.0 < diff[1] < 1e-6
    assert 3.0 < diff[0] / diff[1] < 5.5, diff
