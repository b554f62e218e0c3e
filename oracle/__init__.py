"""Plain FP64 CPU oracle of the polarized Kerr ray tracer (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.

The C++ sources next to this file implement, step by step, the method of
Sec. 2.1 of Moscibrodzka & Yfantis (2023): per pixel a backward null geodesic
with an eps-controlled adaptive step (Sec. 2.2), saved, then covariant fully
polarized transfer of the coherency matrix along it toward the camera, with
synchrotron emission, absorption and Faraday coefficients at every point.
kappa.cpp integrates the coefficients of a kappa electron distribution over
the Lorentz factor (the nonthermal extension); mlp.py is an FP64 reference of
the coefficient surrogate network and its backward pass.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ESCAPED, CAPTURED, STEP_CAP, NONFINITE, AXIS = 0, 1, 2, 3, 4
DIST_KAPPA, DIST_THERMAL = 0, 1
MODEL_ADAF, MODEL_SLAB_PLASMA, MODEL_SLAB_FIXED, MODEL_SNAPSHOT = 0, 1, 2, 3


def build():
    """Compile liboracle.so with the Makefile next to this file."""
    subprocess.run(["make", "-s", "-C", _HERE, "-B"], check=True)


class Camera(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_double), ("incl_deg", ctypes.c_double), ("phi_deg", ctypes.c_double),
        ("r_cam", ctypes.c_double), ("fov_x", ctypes.c_double), ("fov_y", ctypes.c_double),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("freq_hz", ctypes.c_double),
        ("eps", ctypes.c_double), ("max_steps", ctypes.c_int32), ("jitter", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("mass_factor", ctypes.c_int32),
    ]


class Units(ctypes.Structure):
    _fields_ = [("M_bh_g", ctypes.c_double), ("dist_cm", ctypes.c_double)]


class Model(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("n0_cgs", ctypes.c_double), ("T0_K", ctypes.c_double), ("beta", ctypes.c_double),
        ("h_over_r", ctypes.c_double),
        ("slab_radius", ctypes.c_double), ("slab_ne", ctypes.c_double),
        ("slab_thetae", ctypes.c_double), ("slab_B", ctypes.c_double),
        ("slab_bdir", ctypes.c_double * 3), ("slab_jextra", ctypes.c_double * 3),
        ("slab_coef", ctypes.c_double * 8),
        ("electrons", ctypes.c_int32), ("kappa", ctypes.c_double),
        ("update_empty", ctypes.c_int32),
    ]


class Snapshot(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
        ("x1_start", ctypes.c_double), ("dx1", ctypes.c_double),
        ("x2_start", ctypes.c_double), ("dx2", ctypes.c_double),
        ("x3_start", ctypes.c_double), ("dx3", ctypes.c_double),
        ("hslope", ctypes.c_double), ("gamma_ad", ctypes.c_double), ("M_unit_g", ctypes.c_double),
        ("R_high", ctypes.c_double), ("R_low", ctypes.c_double), ("sigma_cut", ctypes.c_double),
        ("r_emit_max", ctypes.c_double), ("prims", ctypes.c_void_p),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_splitmix64.restype = ctypes.c_uint64
        L.or_splitmix64.argtypes = [ctypes.c_uint64]
        L.or_horizon.restype = ctypes.c_double
        L.or_horizon.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_isco.restype = ctypes.c_double
        L.or_isco.argtypes = [ctypes.c_double]
        for name in ("or_metric", "or_metric_inverse", "or_metric_derivs", "or_christoffel"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [ctypes.c_double] * 4 + [_D]
        L.or_pixel_position.argtypes = [ctypes.POINTER(Camera), ctypes.c_int32, ctypes.c_int32,
                                        _D, _D]
        L.or_camera_launch.argtypes = [ctypes.POINTER(Camera), ctypes.c_double, ctypes.c_double,
                                       _D, _D, _D]
        L.or_trace_ray.argtypes = [ctypes.POINTER(Camera), ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]
        L.or_plasma.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Snapshot), ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, _D]
        L.or_thermal_coefficients.restype = None
        L.or_thermal_coefficients.argtypes = [ctypes.c_double] * 5 + [_D]
        L.or_bessel_ratios.restype = None
        L.or_bessel_ratios.argtypes = [ctypes.c_double, _D, _D]
        L.or_mueller_step.restype = None
        L.or_mueller_step.argtypes = [_D, _D, ctypes.c_double, _D]
        L.or_expm.argtypes = [ctypes.c_int, _D, _D]
        L.or_transfer_path.argtypes = [ctypes.POINTER(Camera), ctypes.POINTER(Units),
                                       ctypes.POINTER(Model), ctypes.POINTER(Snapshot),
                                       ctypes.c_double, ctypes.c_double, _D, ctypes.c_int32, _D]
        L.or_render.argtypes = [ctypes.POINTER(Camera), ctypes.POINTER(Units),
                                ctypes.POINTER(Model), ctypes.POINTER(Snapshot), ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64), _D,
                                ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                                ctypes.c_int32]
        L.or_reduce.restype = None
        L.or_reduce.argtypes = [ctypes.POINTER(Camera), ctypes.POINTER(Units), _D, _D, _D]
        L.or_max_threads.restype = ctypes.c_int
        L.or_synchrotron_kernels.restype = None
        L.or_synchrotron_kernels.argtypes = [ctypes.c_int64, _D, _D]
        L.or_bessel_k.restype = None
        L.or_bessel_k.argtypes = [ctypes.c_int64, ctypes.c_double, _D, _D, _D]
        L.or_kappa_integrals.restype = None
        L.or_kappa_integrals.argtypes = [ctypes.c_int32, ctypes.c_int64, _D, _D, ctypes.c_int32]
        L.or_kappa_coefficients.restype = None
        L.or_kappa_coefficients.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 6 + [_D]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_D)


def make_camera(d):
    c = Camera()
    for name, _ in Camera._fields_:
        setattr(c, name, d[name])
    return c


def make_units(d):
    return Units(d["M_bh_g"], d["dist_cm"])


def make_model(d):
    m = Model()
    m.kind = int(d.get("kind", MODEL_ADAF))
    for name in ("n0_cgs", "T0_K", "beta", "h_over_r", "slab_radius", "slab_ne", "slab_thetae",
                 "slab_B"):
        setattr(m, name, float(d.get(name, 0.0)))
    for name, n in (("slab_bdir", 3), ("slab_jextra", 3), ("slab_coef", 8)):
        v = d.get(name, [0.0] * n)
        arr = getattr(m, name)
        for k in range(n):
            arr[k] = float(v[k])
    m.electrons = int(d.get("electrons", 0))
    m.kappa = float(d.get("kappa", 0.0))
    m.update_empty = int(d.get("update_empty", 0))
    return m


class SnapshotHandle:
    """Keeps the primitive array alive while the oracle reads it."""

    def __init__(self, desc, prims):
        self.prims = np.ascontiguousarray(prims, dtype=np.float64)
        assert self.prims.shape == (desc["n1"], desc["n2"], desc["n3"], 8)
        s = Snapshot()
        for name, _ in Snapshot._fields_:
            if name != "prims":
                setattr(s, name, desc[name])
        s.prims = self.prims.ctypes.data
        self.struct = s


def _snap_ptr(snap):
    return ctypes.byref(snap.struct) if snap is not None else None


# ---- building blocks ----

def splitmix64(x):
    return lib().or_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF))


def metric(a, m, r, th):
    out = np.zeros(16)
    lib().or_metric(a, m, r, th, _ptr(out))
    return out.reshape(4, 4)


def metric_inverse(a, m, r, th):
    out = np.zeros(16)
    lib().or_metric_inverse(a, m, r, th, _ptr(out))
    return out.reshape(4, 4)


def metric_derivs(a, m, r, th):
    out = np.zeros(64)
    lib().or_metric_derivs(a, m, r, th, _ptr(out))
    return out.reshape(4, 4, 4)


def christoffel(a, m, r, th):
    out = np.zeros(64)
    lib().or_christoffel(a, m, r, th, _ptr(out))
    return out.reshape(4, 4, 4)


def horizon(a, m=1.0):
    return lib().or_horizon(a, m)


def isco(a):
    return lib().or_isco(a)


def pixel_position(cam, i, j):
    c = make_camera(cam)
    al, be = ctypes.c_double(), ctypes.c_double()
    rc = lib().or_pixel_position(ctypes.byref(c), i, j, ctypes.byref(al), ctypes.byref(be))
    if rc != 0:
        raise ValueError("invalid camera or pixel")
    return al.value, be.value


def camera_launch(cam, alpha, beta):
    c = make_camera(cam)
    X, K, T = np.zeros(4), np.zeros(4), np.zeros(16)
    if lib().or_camera_launch(ctypes.byref(c), alpha, beta, _ptr(X), _ptr(K), _ptr(T)) != 0:
        raise ValueError("invalid camera")
    return X, K, T.reshape(4, 4)


def trace_ray(cam, alpha, beta, cap=None):
    """Returns (path[n_end+1, 8], status)."""
    c = make_camera(cam)
    cap = cam["max_steps"] if cap is None else cap
    buf = np.zeros((cap + 1) * 8)
    n_end, st = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().or_trace_ray(ctypes.byref(c), alpha, beta, cap, _ptr(buf), ctypes.byref(n_end),
                            ctypes.byref(st))
    if rc == -1:
        raise ValueError("invalid camera")
    return buf[: (n_end.value + 1) * 8].reshape(-1, 8).copy(), st.value


def plasma(model, a, m, r, th, ph, L_cm=1.0, snap=None):
    md = make_model(model)
    out = np.zeros(11)
    ok = lib().or_plasma(ctypes.byref(md), _snap_ptr(snap), a, m, r, th, ph, L_cm, _ptr(out))
    return dict(ne=out[0], thetae=out[1], B=out[2], u=out[3:7].copy(), b=out[7:11].copy(),
                valid=bool(ok))


def thermal_coefficients(ne, thetae, B, nu, cos_thb):
    out = np.zeros(8)
    lib().or_thermal_coefficients(ne, thetae, B, nu, cos_thb, _ptr(out))
    return out


def bessel_ratios(x):
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().or_bessel_ratios(x, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def mueller_step(coef, S, w):
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(4)
    lib().or_mueller_step(_ptr(coef), _ptr(S), w, _ptr(out))
    return out


def expm(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    E = np.zeros_like(A)
    if lib().or_expm(n, _ptr(A), _ptr(E)) != 0:
        raise ValueError("expm failed")
    return E


def transfer_path(cam, units, model, alpha, beta, path, snap=None):
    c, u, md = make_camera(cam), make_units(units), make_model(model)
    path = np.ascontiguousarray(path, dtype=np.float64)
    out = np.zeros(4)
    rc = lib().or_transfer_path(ctypes.byref(c), ctypes.byref(u), ctypes.byref(md),
                                _snap_ptr(snap), alpha, beta, _ptr(path), path.shape[0] - 1,
                                _ptr(out))
    if rc != 0:
        raise ValueError("invalid input")
    return out


def render(cam, units, model, snap=None, pixels=None, threads=0):
    """Renders the image (pixels=None) or the listed row-major pixel indices.

    Returns (stokes, status, nsteps): stokes has shape [4, ny, nx] for a whole
    image and [4, npix] for a pixel list."""
    c, u, md = make_camera(cam), make_units(units), make_model(model)
    if pixels is None:
        npix = cam["nx"] * cam["ny"]
        pix_ptr = None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = pixels.shape[0]
        pix_ptr = pixels.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    stokes = np.zeros(4 * npix)
    status = np.zeros(npix, dtype=np.uint8)
    nsteps = np.zeros(npix, dtype=np.int32)
    rc = lib().or_render(ctypes.byref(c), ctypes.byref(u), ctypes.byref(md), _snap_ptr(snap),
                         npix, pix_ptr, _ptr(stokes),
                         status.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                         nsteps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(threads))
    if rc != 0:
        raise ValueError("invalid input")
    if pixels is None:
        return (stokes.reshape(4, cam["ny"], cam["nx"]), status.reshape(cam["ny"], cam["nx"]),
                nsteps.reshape(cam["ny"], cam["nx"]))
    return stokes.reshape(4, npix), status, nsteps


def reduce(cam, units, stokes):
    c, u = make_camera(cam), make_units(units)
    s = np.ascontiguousarray(stokes, dtype=np.float64).reshape(-1)
    flux, imax = np.zeros(4), ctypes.c_double()
    lib().or_reduce(ctypes.byref(c), ctypes.byref(u), _ptr(s), _ptr(flux), ctypes.byref(imax))
    return flux, imax.value


def max_threads():
    return lib().or_max_threads()


def synchrotron_kernels(X):
    """F, G, H of the nonthermal module at the points X: array [n, 3]."""
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    out = np.empty((X.size, 3))
    lib().or_synchrotron_kernels(X.size, _ptr(X), _ptr(out))
    return out


def bessel_k(nu, x):
    """K_nu(x) and int_x^inf K_nu from the oracle's integral representations."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    k = np.empty_like(x)
    ki = np.empty_like(x)
    lib().or_bessel_k(x.size, nu, _ptr(x), _ptr(k), _ptr(ki))
    return k, ki


def kappa_integrals(inputs, dist=DIST_KAPPA, threads=0):
    """The eight dimensionless integrals (I_F, I_G, I_H, A_F, A_G, A_H, R_Q, R_V)
    at rows (kappa, w, X) of inputs: array [n, 8]."""
    a = np.ascontiguousarray(inputs, dtype=np.float64).reshape(-1, 3)
    out = np.empty((a.shape[0], 8))
    lib().or_kappa_integrals(dist, a.shape[0], _ptr(a), _ptr(out), threads)
    return out


def kappa_coefficients(kappa, ne, w, B, nu, cos_thb, dist=DIST_KAPPA):
    """Fluid-frame coefficients (cgs) j_I j_Q j_V a_I a_Q a_V r_Q r_V."""
    out = np.empty(8)
    lib().or_kappa_coefficients(dist, kappa, ne, w, B, nu, cos_thb, _ptr(out))
    return out
