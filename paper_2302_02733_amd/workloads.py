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


def workload(name):
    """Named workloads: returns dict(camera=..., model=..., units=...)."""
    table = {
        # small ADAF image: 64 x 64, the oracle finishes it in seconds
        "adaf64": (adaf_camera(64), ADAF),
        # plain method at scale
        "adaf1024": (adaf_camera(1024), ADAF),
        "adaf4096": (adaf_camera(4096), ADAF),
    }
    cam, model = table[name]
    return {"camera": copy.deepcopy(cam), "model": copy.deepcopy(model),
            "units": copy.deepcopy(UNITS)}


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
