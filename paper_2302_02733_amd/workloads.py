"""Seeded synthetic workloads shared by the GPU path, the oracle and the benchmark.

This module holds parameter sets and seeded input generators only; it contains
none of the method's arithmetic and imports neither the GPU binding nor the
oracle.  The paper's own models (a semianalytic ADAF seen at 60 degrees and a
GRMHD slice seen at 20 degrees, both imaged at 230 GHz; Fig. 1 and Sec. 2.1)
are not available, so these synthetic stand-ins take their shapes.
"""
import copy

M_SUN_G = 1.98841e33
PARSEC_CM = 3.0856775814913673e18

# Sgr A*-like mass and distance (reading: the paper's normalisation is not given).
UNITS = {"M_bh_g": 4.14e6 * M_SUN_G, "dist_cm": 8.127e3 * PARSEC_CM}

# Analytic ADAF-like flow: n0 r^-3/2 exp(-z^2/(2 (0.5 r)^2)), T_e = T0/r,
# beta = 10, Keplerian rotation, toroidal field.
ADAF = {"kind": 0, "n0_cgs": 5e7, "T0_K": 3e11, "beta": 10.0, "h_over_r": 0.5}


def adaf_camera(n, *, jitter=1, seed=1, eps=0.01, max_steps=50000, a=0.9375, incl_deg=60.0,
                freq_hz=230e9, fov=40.0, r_cam=1000.0):
    """Camera of the plain-method ADAF workloads (n x n pixels)."""
    return {
        "a": a, "incl_deg": incl_deg, "phi_deg": 0.0, "r_cam": r_cam,
        "fov_x": fov, "fov_y": fov, "nx": n, "ny": n, "freq_hz": freq_hz, "eps": eps,
        "max_steps": max_steps, "jitter": jitter, "seed": seed, "mass_factor": 1,
    }


def snapshot_camera(n, *, incl_deg=20.0, a=0.94, freq_hz=230e9, eps=0.01, max_steps=50000,
                    fov=40.0, r_cam=1000.0, jitter=0, seed=0):
    """Camera of the snapshot workloads (n x n pixels, no jitter by default)."""
    return {
        "a": a, "incl_deg": incl_deg, "phi_deg": 0.0, "r_cam": r_cam,
        "fov_x": fov, "fov_y": fov, "nx": n, "ny": n, "freq_hz": freq_hz, "eps": eps,
        "max_steps": max_steps, "jitter": jitter, "seed": seed, "mass_factor": 1,
    }


def workload(name):
    """Named workloads: returns dict(camera=..., model=..., units=...) and, for
    snapshot workloads, snapshot=(desc, seed) to be built by make_snapshot."""
    table = {
        # small ADAF image: 64 x 64, the oracle finishes it in seconds
        "adaf64": (adaf_camera(64), ADAF, None),
        # plain method at scale
        "adaf1024": (adaf_camera(1024), ADAF, None),
        "adaf4096": (adaf_camera(4096), ADAF, None),
        # GRMHD-like snapshot 288 x 128 x 128 seen at 20 degrees, 2048 x 2048
        "snap2048": (snapshot_camera(2048), {"kind": 3}, (snapshot_desc(), 7)),
        # small snapshot case for full-image parity
        "snap48": (snapshot_camera(48), {"kind": 3}, (snapshot_desc(48, 32, 32), 7)),
    }
    cam, model, snap = table[name]
    out = {"camera": copy.deepcopy(cam), "model": copy.deepcopy(model),
           "units": copy.deepcopy(UNITS)}
    if snap is not None:
        out["snapshot"] = (copy.deepcopy(snap[0]), snap[1])
    return out


def flat_camera(nx=2, ny=2, fov=8.0, r_cam=1000.0, incl_deg=90.0, eps=0.01, freq_hz=230e9,
                max_steps=50000):
    """Flat-space test camera (mass factor 0, a = 0)."""
    return {
        "a": 0.0, "incl_deg": incl_deg, "phi_deg": 0.0, "r_cam": r_cam,
        "fov_x": fov, "fov_y": fov, "nx": nx, "ny": ny, "freq_hz": freq_hz, "eps": eps,
        "max_steps": max_steps, "jitter": 0, "seed": 0, "mass_factor": 0,
    }


def pixel_sample(nx, ny, count, seed):
    """Seeded sample of distinct row-major pixel indices (sorted)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    count = min(count, nx * ny)
    return np.sort(rng.choice(nx * ny, size=count, replace=False)).astype(np.int64)


# ---------------------------------------------------------------------------
# Synthetic GRMHD-like snapshot on a modified Kerr-Schild grid: a torus
# profile with seeded power-law Gaussian random fluctuations (a stand-in for
# the paper's GRMHD slice, which is not available).  Primitives (rho, u, U1,
# U2, U3, B1, B2, B3) in code units, layout [n1][n2][n3][8].  The code-unit
# density scale is set so that the mass unit 1e19 g puts the 230 GHz flux of
# the 288 x 128 x 128 snapshot seen at 20 degrees at 2.4 Jy (Sgr A*-like, the
# way GRMHD images are normalised); mass units 1e17 to 1e20 g then run from
# optically thin to thick.
# ---------------------------------------------------------------------------

def snapshot_desc(n1=288, n2=128, n3=128, r_in=1.2, r_out=1000.0, hslope=0.3, M_unit_g=1e19,
                  R_high=40.0, R_low=1.0, sigma_cut=1.0, r_emit_max=50.0, gamma_ad=13.0 / 9.0):
    import math
    return {
        "n1": n1, "n2": n2, "n3": n3,
        "x1_start": math.log(r_in), "dx1": (math.log(r_out) - math.log(r_in)) / n1,
        "x2_start": 0.0, "dx2": 1.0 / n2, "x3_start": 0.0, "dx3": 2.0 * math.pi / n3,
        "hslope": hslope, "gamma_ad": gamma_ad, "M_unit_g": M_unit_g, "R_high": R_high,
        "R_low": R_low, "sigma_cut": sigma_cut, "r_emit_max": r_emit_max,
    }


def _gaussian_field(shape, rng, slope=-11.0 / 3.0):
    """Periodic zero-mean unit-variance Gaussian random field with power
    spectrum P(k) ~ k^slope on the index grid (slope -11/3: Kolmogorov)."""
    import numpy as np
    k = [np.fft.fftfreq(n) * n for n in shape]
    K2 = k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2
    amp = np.zeros_like(K2)
    nz = K2 > 0
    amp[nz] = K2[nz] ** (slope / 4.0)
    noise = rng.standard_normal(shape)
    f = np.fft.ifftn(np.fft.fftn(noise) * amp).real
    f -= f.mean()
    return f / f.std()


def make_snapshot(desc, seed=7, a=0.94):
    """Seeded synthetic snapshot for `desc`; returns float64 [n1][n2][n3][8]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    n1, n2, n3 = desc["n1"], desc["n2"], desc["n3"]
    x1 = desc["x1_start"] + (np.arange(n1) + 0.5) * desc["dx1"]
    x2 = desc["x2_start"] + (np.arange(n2) + 0.5) * desc["dx2"]
    h = desc["hslope"]
    r = np.exp(x1)[:, None, None]
    th = (np.pi * x2 + 0.5 * (1 - h) * np.sin(2 * np.pi * x2))[None, :, None]
    rh = 1.0 + np.sqrt(1.0 - a * a)
    rho = np.exp(-(r - 15.0) ** 2 / (2 * 6.0 ** 2) - np.cos(th) ** 2 / (2 * 0.3 ** 2)) + 1e-4 * (r / 15.0) ** -1.5
    uu = 0.2 * rho / r
    d = [_gaussian_field((n1, n2, n3), rng) for _ in range(5)]
    P = np.zeros((n1, n2, n3, 8))
    P[..., 0] = rho * np.exp(0.5 * d[0] - 0.125)
    P[..., 1] = uu * np.exp(0.5 * d[1] - 0.125)
    vK = 1.0 / (r ** 1.5 + a)                                   # angular-velocity scale
    P[..., 2] = (-0.02 / np.sqrt(r) + 0.05 * np.sqrt(1.0 / r) * d[2]) / r      # U1 (per unit x1)
    P[..., 3] = 0.05 * vK * d[3] / np.pi                        # U2 (per unit x2)
    P[..., 4] = vK * np.ones_like(d[4])                          # U3 (angular)
    btor = np.sqrt(2 * (desc["gamma_ad"] - 1) * uu / 10.0)
    P[..., 5] = 0.1 * np.sign(np.cos(th)) * (rh / r) ** 2 / r * (1 + 0.3 * d[4])
    P[..., 7] = btor / (r * np.maximum(np.sin(th), 1e-3)) * (1 + 0.3 * d[4])
    # density scale 10^1.5 in code units: rho, u scale with it, B with its root
    P[..., 0:2] *= 10 ** 1.5
    P[..., 5:8] *= 10 ** 0.75
    return np.ascontiguousarray(P)


# ---------------------------------------------------------------------------
# Batched image library on the snapshot: instances drawn with SplitMix64
# (seed 11): mass unit 10^U(17,20) g, R_high in {1, 10, 40, 160}, inclination
# in {20, 60, 120, 160} deg, frequency in {86, 230, 345} GHz, resolution in
# {128, 256, 512, 1024}; geodesics are shared by the instances of one
# (inclination, resolution) group.
# ---------------------------------------------------------------------------

_MASK64 = (1 << 64) - 1


def _splitmix64(seed):
    state = seed & _MASK64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        yield z ^ (z >> 31)


def batch_library(n_inst=256, seed=11, resolutions=(128, 256, 512, 1024)):
    """Returns (groups, instances): groups are snapshot cameras, one per
    (inclination, resolution) in order of first appearance; instances are dicts
    with group, freq_hz, M_unit_g, R_high."""
    rng = _splitmix64(seed)

    def u01():
        return (next(rng) >> 11) * 2.0 ** -53

    def choice(seq):
        return seq[min(int(u01() * len(seq)), len(seq) - 1)]

    groups, index, instances = [], {}, []
    for _ in range(n_inst):
        m_unit = 10.0 ** (17.0 + 3.0 * u01())
        r_high = choice((1.0, 10.0, 40.0, 160.0))
        incl = choice((20.0, 60.0, 120.0, 160.0))
        freq = choice((86e9, 230e9, 345e9))
        n = choice(tuple(resolutions))
        key = (incl, n)
        if key not in index:
            index[key] = len(groups)
            groups.append(snapshot_camera(n, incl_deg=incl))
        instances.append({"group": index[key], "freq_hz": freq, "M_unit_g": m_unit, "R_high": r_high})
    return groups, instances


def kappa_inputs(n, seed):
    """Seeded inputs of the kappa-coefficient surrogate: rows (kappa, w, X,
    cos theta_B) with kappa ~ U[3, 8], log10 w ~ U[-0.5, 2], log10 X ~ U[-2, 7],
    theta_B ~ U[0, pi] (the box the network covers)."""
    import numpy as np
    r = np.random.Generator(np.random.PCG64(seed))
    kap = r.uniform(3.0, 8.0, n)
    w = 10.0 ** r.uniform(-0.5, 2.0, n)
    X = 10.0 ** r.uniform(-2.0, 7.0, n)
    cth = np.cos(r.uniform(0.0, np.pi, n))
    return np.stack([kap, w, X, cth], axis=1)
