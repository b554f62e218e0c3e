"""Thin ctypes binding of libkrt.so (include/krt.h).

Argument marshalling only: every step of the ray-tracing path runs in the HIP
kernels of libkrt.so.  PyTorch provides device memory and the stream.  The
binding fails loudly when the library is missing; there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# KRT_LIBRARY selects another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("KRT_LIBRARY") or os.path.join(_HERE, "libkrt.so")

OK, E_INVAL, E_NOMEM, E_HIP, E_STATE, E_UNSUPPORTED = range(6)
RAY_ESCAPED, RAY_CAPTURED, RAY_STEP_CAP, RAY_NONFINITE, RAY_AXIS = range(5)


class KrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"krt error {code}: {msg}")
        self.code = code


class Camera(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("a", ctypes.c_double), ("incl_deg", ctypes.c_double),
        ("phi_deg", ctypes.c_double), ("r_cam", ctypes.c_double), ("fov_x", ctypes.c_double),
        ("fov_y", ctypes.c_double), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("freq_hz", ctypes.c_double), ("eps", ctypes.c_double), ("max_steps", ctypes.c_int32),
        ("jitter", ctypes.c_int32), ("seed", ctypes.c_uint64), ("mass_factor", ctypes.c_int32),
    ]


class Units(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("M_bh_g", ctypes.c_double),
                ("dist_cm", ctypes.c_double)]


class Adaf(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n0_cgs", ctypes.c_double),
                ("T0_K", ctypes.c_double), ("beta", ctypes.c_double),
                ("h_over_r", ctypes.c_double), ("field_geom", ctypes.c_int32)]


class SnapshotDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
        ("n3", ctypes.c_int32), ("x1_start", ctypes.c_double), ("dx1", ctypes.c_double),
        ("x2_start", ctypes.c_double), ("dx2", ctypes.c_double), ("x3_start", ctypes.c_double),
        ("dx3", ctypes.c_double), ("hslope", ctypes.c_double), ("gamma_ad", ctypes.c_double),
        ("M_unit_g", ctypes.c_double), ("R_high", ctypes.c_double), ("R_low", ctypes.c_double),
        ("sigma_cut", ctypes.c_double), ("r_emit_max", ctypes.c_double), ("layout", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("rays", ctypes.c_int64),
                ("total_steps", ctypes.c_int64), ("status_count", ctypes.c_int64 * 5),
                ("max_steps_seen", ctypes.c_int32), ("long_rays", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double * 2), ("surrogate_points", ctypes.c_int64),
                ("exact_points", ctypes.c_int64)]

    def as_dict(self):
        return {"rays": self.rays, "total_steps": self.total_steps,
                "status_count": list(self.status_count), "max_steps_seen": self.max_steps_seen,
                "long_rays": self.long_rays, "kernel_ms": list(self.kernel_ms),
                "surrogate_points": self.surrogate_points, "exact_points": self.exact_points}


class LaunchConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("tile_w", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("path_cap", ctypes.c_int32),
                ("order", ctypes.c_int32)]

    def as_dict(self):
        return {"tile_w": self.tile_w, "blocks_per_cu": self.blocks_per_cu,
                "path_cap": self.path_cap, "order": self.order}


class TrainConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("set_norm", ctypes.c_int32), ("lr_max", ctypes.c_double), ("lr_min", ctypes.c_double),
                ("warmup_frac", ctypes.c_double), ("seed", ctypes.c_uint64)]


class Instance(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("group", ctypes.c_int32),
                ("freq_hz", ctypes.c_double), ("M_unit_g", ctypes.c_double),
                ("R_high", ctypes.c_double), ("d_stokes", ctypes.c_void_p),
                ("d_status", ctypes.c_void_p)]


# Every symbol include/krt.h declares, with (restype, argtypes).
_P = ctypes.c_void_p
_SIGS = {
    "krt_abi_version": (ctypes.c_int, []),
    "krt_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)]),
    "krt_destroy": (ctypes.c_int, [_P]),
    "krt_set_stream": (ctypes.c_int, [_P, _P]),
    "krt_set_units": (ctypes.c_int, [_P, ctypes.POINTER(Units)]),
    "krt_set_model_adaf": (ctypes.c_int, [_P, ctypes.POINTER(Adaf)]),
    "krt_set_model_snapshot": (ctypes.c_int, [_P, ctypes.POINTER(SnapshotDesc), _P, ctypes.c_int]),
    "krt_trace": (ctypes.c_int, [_P, ctypes.POINTER(Camera), _P, _P, ctypes.POINTER(Stats)]),
    "krt_trace_steps": (ctypes.c_int, [_P, ctypes.POINTER(Camera), _P, _P, _P, ctypes.POINTER(Stats)]),
    "krt_probe_fma": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double)]),
    "krt_trace_probe": (ctypes.c_int, [_P, ctypes.POINTER(Camera), _P, ctypes.c_int32, _P,
                                       ctypes.POINTER(Stats)]),
    "krt_reduce": (ctypes.c_int, [_P, _P, ctypes.POINTER(Camera), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]),
    "krt_reduce_noalloc": (ctypes.c_int, [_P, _P, ctypes.POINTER(Camera), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
    "krt_last_error": (ctypes.c_char_p, [_P]),
    "krt_check_camera": (ctypes.c_int, [ctypes.POINTER(Camera), ctypes.c_char_p, ctypes.c_size_t]),
    "krt_geodesic_only": (ctypes.c_int, [_P, ctypes.POINTER(Camera), _P, _P, _P, _P]),
    "krt_plasma_eval": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _P, _P]),
    "krt_coeffs": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
    "krt_bessel_ratios": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
    "krt_mueller_step": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, ctypes.c_double, _P]),
    "krt_set_precision": (ctypes.c_int, [_P, ctypes.c_int]),
    "krt_set_launch_config": (ctypes.c_int, [_P, ctypes.POINTER(LaunchConfig)]),
    "krt_get_launch_config": (ctypes.c_int, [_P, ctypes.POINTER(LaunchConfig)]),
    "krt_trace_batch": (ctypes.c_int, [_P, ctypes.POINTER(Camera), ctypes.c_int32, ctypes.POINTER(Instance),
                                       ctypes.c_int32, ctypes.POINTER(Stats)]),
    "krt_autotune": (ctypes.c_int, [_P, ctypes.POINTER(Camera), ctypes.c_int32, ctypes.POINTER(Instance),
                                    ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(LaunchConfig)]),
    "krt_set_electrons": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double]),
    "krt_kappa_integrals": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
    "krt_mueller_general": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, ctypes.c_double, _P]),
    "krt_mlp_set_params": (ctypes.c_int, [_P, _P, _P]),
    "krt_mlp_get_params": (ctypes.c_int, [_P, _P, _P]),
    "krt_mlp_init": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "krt_mlp_grad": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "krt_mlp_train": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, ctypes.POINTER(TrainConfig),
                                     ctypes.POINTER(ctypes.c_double)]),
    "krt_mlp_eval": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
}

MLP_PARAMS = 9160
MLP_NORM = 176
ELECTRONS_THERMAL, ELECTRONS_KAPPA_EXACT, ELECTRONS_KAPPA_SURROGATE = 0, 1, 2

PRECISION_FP64 = 0
PRECISION_FP32_TRANSFER = 1
DTYPE_F64 = 0
DTYPE_F32 = 1

_lib = None


def lib():
    """Loads libkrt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2302_02733_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def make_camera(d):
    c = Camera()
    c.struct_size = ctypes.sizeof(Camera)
    for name, _ in Camera._fields_[1:]:
        setattr(c, name, d[name])
    return c


def check_camera(d):
    """Host-only validation; returns '' when valid, else the message."""
    c = make_camera(d)
    buf = ctypes.create_string_buffer(256)
    rc = lib().krt_check_camera(ctypes.byref(c), buf, 256)
    return "" if rc == OK else buf.value.decode()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, device):
    if t.device != device:
        raise ValueError(f"tensor on {t.device}, context on {device}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t


class Context:
    """One library context on one HIP device."""

    def __init__(self, device=0):
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = lib().krt_create(device, ctypes.byref(h))
        if rc != OK:
            raise KrtError(rc, "krt_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().krt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise KrtError(rc, lib().krt_last_error(self.h).decode())

    def _stream(self):
        s = torch.cuda.current_stream(self.device)
        self._check(lib().krt_set_stream(self.h, ctypes.c_void_p(s.cuda_stream)))

    def set_units(self, d):
        u = Units(ctypes.sizeof(Units), d["M_bh_g"], d["dist_cm"])
        self._check(lib().krt_set_units(self.h, ctypes.byref(u)))

    def set_model_adaf(self, d):
        m = Adaf(ctypes.sizeof(Adaf), d["n0_cgs"], d["T0_K"], d["beta"], d["h_over_r"],
                 int(d.get("field_geom", 0)))
        self._check(lib().krt_set_model_adaf(self.h, ctypes.byref(m)))

    def set_model_snapshot(self, desc, prims):
        """desc: snapshot description dict (layout 0 or 1); prims: float64 or
        float32 device tensor [n1][n2][n3][8] (layout 0) or [8][n1][n2][n3]
        (layout 1), borrowed (keep it alive while the model is in use)."""
        _dev(prims, self.device)
        n = (desc["n1"], desc["n2"], desc["n3"])
        shape = (8,) + n if desc.get("layout", 0) == 1 else n + (8,)
        if prims.dtype not in (torch.float64, torch.float32) or tuple(prims.shape) != shape:
            raise ValueError(f"prims must be float64 or float32 {list(shape)}")
        d = SnapshotDesc()
        d.struct_size = ctypes.sizeof(SnapshotDesc)
        for name, _ in SnapshotDesc._fields_[1:]:
            setattr(d, name, desc.get(name, 0))
        self._snapshot = prims
        dtype = DTYPE_F64 if prims.dtype == torch.float64 else DTYPE_F32
        self._check(lib().krt_set_model_snapshot(self.h, ctypes.byref(d), _ptr(prims), dtype))

    def set_launch_config(self, tile_w=8, blocks_per_cu=0, path_cap=0, order=1):
        c = LaunchConfig(ctypes.sizeof(LaunchConfig), tile_w, blocks_per_cu, path_cap, order)
        self._check(lib().krt_set_launch_config(self.h, ctypes.byref(c)))

    def get_launch_config(self):
        c = LaunchConfig()
        self._check(lib().krt_get_launch_config(self.h, ctypes.byref(c)))
        return c.as_dict()

    def _batch_args(self, groups, instances):
        cams = (Camera * len(groups))(*[make_camera(g) for g in groups])
        arr = (Instance * len(instances))()
        for k, d in enumerate(instances):
            g = groups[d["group"]]
            st = d["stokes"]
            _dev(st, self.device)
            if st.dtype != torch.float64 or tuple(st.shape) != (4, g["ny"], g["nx"]):
                raise ValueError("instance stokes must be float64 [4][ny][nx] of its group")
            status = d.get("status")
            if status is not None:
                _dev(status, self.device)
                if status.dtype != torch.uint8 or tuple(status.shape) != (g["ny"], g["nx"]):
                    raise ValueError("instance status must be uint8 [ny][nx]")
            arr[k] = Instance(ctypes.sizeof(Instance), d["group"], d["freq_hz"], d.get("M_unit_g", 0.0),
                              d.get("R_high", 0.0), st.data_ptr(),
                              status.data_ptr() if status is not None else None)
        return cams, arr

    def trace_batch(self, groups, instances, stats=True):
        """groups: camera dicts (shared geodesics); instances: dicts with group,
        freq_hz, M_unit_g, R_high (snapshot; 0 = the model's), stokes
        ([4][ny][nx] float64 device tensor) and optionally status."""
        cams, arr = self._batch_args(groups, instances)
        self._stream()
        s = Stats()
        s.struct_size = ctypes.sizeof(Stats)
        self._check(lib().krt_trace_batch(self.h, cams, len(groups), arr, len(instances),
                                          ctypes.byref(s) if stats else None))
        return s.as_dict() if stats else None

    def autotune(self, groups, instances, cache_path=None):
        cams, arr = self._batch_args(groups, instances)
        self._stream()
        c = LaunchConfig()
        self._check(lib().krt_autotune(self.h, cams, len(groups), arr, len(instances),
                                       cache_path.encode() if cache_path else None, ctypes.byref(c)))
        return c.as_dict()

    def set_precision(self, precision):
        """PRECISION_FP64 or PRECISION_FP32_TRANSFER (FP32 transfer operators,
        FP64 geodesics and FP64 transfer state)."""
        self._check(lib().krt_set_precision(self.h, int(precision)))

    def set_model(self, d, prims=None):
        kind = int(d.get("kind", 0))
        if kind == 0:
            return self.set_model_adaf(d)
        if kind == 3:
            return self.set_model_snapshot(d, prims)
        raise ValueError(f"unsupported model kind {kind}")

    def trace(self, cam, stokes=None, status=None, nsteps=None, stats=True):
        """Traces the image; returns dict(stokes [4,ny,nx] f64, status [ny,nx] u8,
        nsteps [ny,nx] i32 or None, stats dict or None)."""
        nx, ny = cam["nx"], cam["ny"]
        if stokes is None:
            stokes = torch.empty((4, ny, nx), dtype=torch.float64, device=self.device)
        if status is None:
            status = torch.empty((ny, nx), dtype=torch.uint8, device=self.device)
        for t, shape, dt in ((stokes, (4, ny, nx), torch.float64), (status, (ny, nx), torch.uint8)):
            _dev(t, self.device)
            if tuple(t.shape) != shape or t.dtype != dt:
                raise ValueError("bad output tensor")
        if nsteps is not None:
            _dev(nsteps, self.device)
            if tuple(nsteps.shape) != (ny, nx) or nsteps.dtype != torch.int32:
                raise ValueError("bad nsteps tensor")
        c = make_camera(cam)
        st = Stats()
        st.struct_size = ctypes.sizeof(Stats)
        self._stream()
        self._check(lib().krt_trace_steps(self.h, ctypes.byref(c), _ptr(stokes), _ptr(status),
                                          _ptr(nsteps), ctypes.byref(st) if stats else None))
        return {"stokes": stokes, "status": status, "nsteps": nsteps,
                "stats": st.as_dict() if stats else None}

    def trace_probe(self, cam, pixels, stokes=None):
        """Measurement probe: every listed row-major pixel of the camera's image
        traced by the 64 lanes of one wave (no lane divergence).  Returns
        dict(stokes [4, npix] f64, stats dict)."""
        import numpy as np
        pix = np.ascontiguousarray(pixels, dtype=np.int32)
        n = int(pix.shape[0])
        if stokes is None:
            stokes = torch.empty((4, n), dtype=torch.float64, device=self.device)
        _dev(stokes, self.device)
        if tuple(stokes.shape) != (4, n) or stokes.dtype != torch.float64:
            raise ValueError("bad output tensor")
        c = make_camera(cam)
        st = Stats()
        st.struct_size = ctypes.sizeof(Stats)
        self._stream()
        self._check(lib().krt_trace_probe(self.h, ctypes.byref(c), pix.ctypes.data_as(_P), n, _ptr(stokes),
                                          ctypes.byref(st)))
        return {"stokes": stokes, "stats": st.as_dict()}

    def probe_fma(self, blocks, iters, chains=8):
        """FP64 FMA issue probe; returns the kernel time in ms (FMAs performed:
        blocks x 256 x iters x 16 x chains)."""
        ms = ctypes.c_double(0.0)
        self._stream()
        self._check(lib().krt_probe_fma(self.h, int(blocks), int(iters), int(chains), ctypes.byref(ms)))
        return ms.value

    def reduce(self, stokes, cam):
        """Returns (flux_jy[4], I_max); synchronises."""
        _dev(stokes, self.device)
        c = make_camera(cam)
        flux = (ctypes.c_double * 4)()
        imax = ctypes.c_double()
        self._stream()
        self._check(lib().krt_reduce(self.h, _ptr(stokes), ctypes.byref(c), flux, ctypes.byref(imax)))
        return list(flux), imax.value

    def geodesic_only(self, cam, drift=False):
        """Returns (end state [ny,nx,8], steps [ny,nx], status [ny,nx]) and,
        with drift=True, also the invariant drift [ny,nx,4] (E, L, Q, null)."""
        nx, ny = cam["nx"], cam["ny"]
        end = torch.empty((ny, nx, 8), dtype=torch.float64, device=self.device)
        ns = torch.empty((ny, nx), dtype=torch.int32, device=self.device)
        st = torch.empty((ny, nx), dtype=torch.uint8, device=self.device)
        dr = torch.empty((ny, nx, 4), dtype=torch.float64, device=self.device) if drift else None
        c = make_camera(cam)
        self._stream()
        self._check(lib().krt_geodesic_only(self.h, ctypes.byref(c), _ptr(end), _ptr(ns), _ptr(st), _ptr(dr)))
        return (end, ns, st, dr) if drift else (end, ns, st)

    def plasma_eval(self, X, a, mass_factor=1):
        X = _dev(X, self.device)
        out = torch.empty((X.shape[0], 12), dtype=torch.float64, device=self.device)
        self._stream()
        self._check(lib().krt_plasma_eval(self.h, X.shape[0], a, mass_factor, _ptr(X), _ptr(out)))
        return out

    def coeffs(self, inp):
        inp = _dev(inp, self.device)
        out = torch.empty((inp.shape[0], 8), dtype=torch.float64, device=self.device)
        self._stream()
        self._check(lib().krt_coeffs(self.h, inp.shape[0], _ptr(inp), _ptr(out)))
        return out

    def bessel_ratios(self, x):
        x = _dev(x, self.device)
        out = torch.empty((x.shape[0], 2), dtype=torch.float64, device=self.device)
        self._stream()
        self._check(lib().krt_bessel_ratios(self.h, x.shape[0], _ptr(x), _ptr(out)))
        return out

    def mueller_step(self, coef, S, w):
        coef, S = _dev(coef, self.device), _dev(S, self.device)
        out = torch.empty_like(S)
        self._stream()
        self._check(lib().krt_mueller_step(self.h, coef.shape[0], _ptr(coef), _ptr(S), float(w), _ptr(out)))
        return out

    # ---- nonthermal electrons and the learned surrogate ----
    def set_electrons(self, kind, kappa=5.0):
        """ELECTRONS_THERMAL, ELECTRONS_KAPPA_EXACT or ELECTRONS_KAPPA_SURROGATE."""
        self._check(lib().krt_set_electrons(self.h, int(kind), float(kappa)))

    def kappa_integrals(self, inp):
        """inp [n, 3] float64 device (kappa, w, X) -> [n, 8] integrals."""
        inp = _dev(inp, self.device)
        if inp.dtype != torch.float64 or inp.dim() != 2 or inp.shape[1] != 3:
            raise ValueError("inputs must be float64 [n, 3]")
        out = torch.empty((inp.shape[0], 8), dtype=torch.float64, device=self.device)
        self._stream()
        self._check(lib().krt_kappa_integrals(self.h, inp.shape[0], _ptr(inp), _ptr(out)))
        return out

    def mueller_general(self, coef, S, w):
        coef, S = _dev(coef, self.device), _dev(S, self.device)
        if coef.shape[1] != 8 or S.shape[1] != 4:
            raise ValueError("coef [n, 8] and S [n, 4]")
        out = torch.empty_like(S)
        self._stream()
        self._check(lib().krt_mueller_general(self.h, coef.shape[0], _ptr(coef), _ptr(S), float(w), _ptr(out)))
        return out

    def mlp_set_params(self, params, norm):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        nm = np.ascontiguousarray(norm, dtype=np.float64)
        if p.size != MLP_PARAMS or nm.size != MLP_NORM:
            raise ValueError(f"params must hold {MLP_PARAMS} floats and norm {MLP_NORM} doubles")
        self._stream()
        self._check(lib().krt_mlp_set_params(self.h, p.ctypes.data_as(_P), nm.ctypes.data_as(_P)))

    def mlp_get_params(self):
        import numpy as np
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        nm = np.empty(MLP_NORM, dtype=np.float64)
        self._stream()
        self._check(lib().krt_mlp_get_params(self.h, p.ctypes.data_as(_P), nm.ctypes.data_as(_P)))
        return p, nm

    def mlp_init(self, seed):
        self._stream()
        self._check(lib().krt_mlp_init(self.h, int(seed)))

    def _set_check(self, inp, integ):
        inp, integ = _dev(inp, self.device), _dev(integ, self.device)
        if inp.dtype != torch.float64 or integ.dtype != torch.float64 or inp.dim() != 2 or inp.shape[1] != 4 \
                or tuple(integ.shape) != (inp.shape[0], 8):
            raise ValueError("inputs float64 [n, 4] and integrals float64 [n, 8]")
        return inp, integ

    def mlp_grad(self, inp, integ):
        """Gradient of the standardised mean-square loss; returns (grad [9160] f32 tensor, loss)."""
        inp, integ = self._set_check(inp, integ)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._stream()
        self._check(lib().krt_mlp_grad(self.h, inp.shape[0], _ptr(inp), _ptr(integ), _ptr(g), ctypes.byref(loss)))
        return g, loss.value

    def mlp_train(self, inp, integ, epochs, batch=16384, lr_max=3e-3, lr_min=1e-6, warmup_frac=0.03, seed=1,
                  set_norm=True):
        inp, integ = self._set_check(inp, integ)
        c = TrainConfig(ctypes.sizeof(TrainConfig), int(epochs), int(batch), 1 if set_norm else 0,
                        float(lr_max), float(lr_min), float(warmup_frac), int(seed))
        loss = ctypes.c_double()
        self._stream()
        self._check(lib().krt_mlp_train(self.h, inp.shape[0], _ptr(inp), _ptr(integ), ctypes.byref(c),
                                        ctypes.byref(loss)))
        return loss.value

    def mlp_eval(self, inp):
        """inp [n, 4] float64 (kappa, w, X, cos theta) -> [n, 8] integrals (bf16 MFMA)."""
        inp = _dev(inp, self.device)
        if inp.dtype != torch.float64 or inp.dim() != 2 or inp.shape[1] != 4:
            raise ValueError("inputs must be float64 [n, 4]")
        out = torch.empty((inp.shape[0], 8), dtype=torch.float64, device=self.device)
        self._stream()
        self._check(lib().krt_mlp_eval(self.h, inp.shape[0], _ptr(inp), _ptr(out)))
        return out
