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
