"""ctypes binding of the C ABI declared in include/lbm.h (liblbm.so).

Argument marshalling only: every step of the method runs in the HIP kernels of
liblbm.so.  The functions keep the C names; ``Lattice`` is a thin convenience
wrapper used by the tests and the benchmark.  If the shared library has not
been built, loading fails loudly -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbm.so")

LBM_OK, LBM_E_ARG, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_STATE, LBM_E_NONFINITE, LBM_E_NO_CONTACT_LINE, \
    LBM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_F32, LBM_F64, LBM_F32_MIXED = 0, 1, 2
LBM_PERIODIC, LBM_WALL = 0, 1
LBM_MRT, LBM_BGK = 0, 1
LBM_BC_HALFWAY, LBM_BC_BOUZIDI_MC = 0, 1
LBM_MODEL_CHEMICAL_POTENTIAL, LBM_MODEL_PSEUDOPOTENTIAL, LBM_MODEL_PHASE_FIELD = 0, 1, 2
LBM_STEP_AUTO, LBM_STEP_SPLIT = 0, 1
LBM_SOLID_SPHERE = 0
LBM_SOLID_CAVITY = 1
LBM_WET_UNIFORM, LBM_WET_STRIPES = 0, 1
FIELD_RHO, FIELD_F, FIELD_VEL, FIELD_MU, FIELD_CLASS, FIELD_MASS, FIELD_PHI, FIELD_G = range(8)
MAX_SECTORS = 64


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


class lbm_config(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("precision", C.c_int), ("n", C.c_int * 3), ("axis_bc", C.c_int * 3),
        ("collision", C.c_int), ("bc_mode", C.c_int),
        ("tau", C.c_double), ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
        ("s_pi", C.c_double), ("s_m", C.c_double), ("Tr", C.c_double),
        ("pr_a", C.c_double), ("pr_b", C.c_double), ("pr_R", C.c_double), ("pr_omega", C.c_double),
        ("k", C.c_double), ("kappa", C.c_double), ("g", C.c_double * 3), ("g_start_step", C.c_int64),
        ("rho_l", C.c_double), ("rho_g", C.c_double), ("wall_mu", C.c_double), ("stream", C.c_void_p),
        ("model", C.c_int), ("sc_G", C.c_double), ("step_kernel", C.c_int),
        ("pf_A", C.c_double), ("pf_kappa", C.c_double), ("pf_gamma", C.c_double), ("pf_tau", C.c_double),
        ("pf_rho0", C.c_double),
    ]


class lbm_solid(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("wet_mode", C.c_int), ("center", C.c_double * 3), ("radius", C.c_double),
        ("mu_w", C.c_double), ("mu_w2", C.c_double), ("stripe_width", C.c_double), ("pole", C.c_double * 3),
    ]


class lbm_drop(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("radius", C.c_double)]


class lbm_measure_opts(C.Structure):
    _fields_ = [("solid_index", C.c_int), ("n_sectors", C.c_int), ("rho_m", C.c_double)]


class lbm_angle(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("status", C.c_int32), ("n_sectors", C.c_int32), ("n_valid", C.c_int32),
        ("pad_", C.c_int32), ("mean_deg", C.c_double), ("adv_deg", C.c_double), ("rec_deg", C.c_double),
        ("axis", C.c_double * 3), ("sector_deg", C.c_double * MAX_SECTORS),
        ("contact", (C.c_double * 3) * MAX_SECTORS),
    ]

    def sectors(self):
        return np.array(self.sector_deg[: self.n_sectors])


class lbm_young_opts(C.Structure):
    _fields_ = [("gamma", C.c_double), ("theta1_deg", C.c_double), ("theta2_deg", C.c_double),
                ("roughness", C.c_double), ("band_lo", C.c_double), ("band_hi", C.c_double)]


class lbm_young(C.Structure):
    _fields_ = [("step", C.c_int64), ("status", C.c_int32), ("n_sectors", C.c_int32),
                ("count", (C.c_int32 * 2) * MAX_SECTORS), ("phi_d", C.c_double * MAX_SECTORS),
                ("theta_eq_deg", C.c_double * MAX_SECTORS), ("force", C.c_double * MAX_SECTORS)]


class lbm_info(C.Structure):
    _fields_ = [
        ("Tc", C.c_double), ("T", C.c_double), ("alpha", C.c_double), ("rho_g", C.c_double),
        ("rho_l", C.c_double), ("mu_sat", C.c_double), ("p_sat", C.c_double), ("wall_mu", C.c_double),
        ("rho_m", C.c_double), ("Q", C.c_int32), ("precision", C.c_int32), ("N", C.c_int64),
        ("step", C.c_int64), ("n_fluid", C.c_int64), ("n_layer1", C.c_int64), ("n_layer2", C.c_int64),
        ("n_boundary", C.c_int64),
    ]


class lbm_case(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("solid", lbm_solid), ("drop", lbm_drop)]


class lbm_batch_opts(C.Structure):
    _fields_ = [("autotune", C.c_int), ("tile_w", C.c_int), ("blocks_per_cu", C.c_int), ("cache_path", C.c_char_p)]


class lbm_unet_config(C.Structure):
    _fields_ = [("H", C.c_int), ("W", C.c_int), ("batch", C.c_int), ("in_channels", C.c_int),
                ("base_channels", C.c_int), ("levels", C.c_int), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("stream", C.c_void_p)]


LBM_UNET_WEIGHTS, LBM_UNET_GRADS = 0, 1


class lbm_batch_info(C.Structure):
    _fields_ = [("total_nodes", C.c_int64), ("fluid_nodes", C.c_int64), ("ncases", C.c_int32), ("tile_w", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("n_items", C.c_int32), ("tune_ms_per_step", C.c_double),
                ("step", C.c_int64), ("rho_g", C.c_double), ("rho_l", C.c_double)]


_lib = None

# exported symbols of include/lbm.h (the binding and the tests check them)
EXPORTS = ("lbm_config_default", "lbm_create", "lbm_destroy", "lbm_set_solid", "lbm_init_drops",
           "lbm_step", "lbm_set_measure", "lbm_measure_angle", "lbm_read", "lbm_write", "lbm_sync",
           "lbm_get_info", "lbm_profile_step", "lbm_young_force", "lbm_set_young", "lbm_young_series",
           "lbm_last_error", "lbm_measure_field", "lbm_batch_create",
           "lbm_batch_destroy",
           "lbm_batch_step", "lbm_batch_sync", "lbm_batch_angles", "lbm_batch_measure", "lbm_batch_young_force",
           "lbm_batch_set_young", "lbm_batch_young_last",
           "lbm_batch_read", "lbm_batch_write", "lbm_batch_get_info", "lbm_batch_tune", "lbm_batch_profile_step", "lbm_batch_last_error",
           "lbm_unet_config_default", "lbm_unet_create", "lbm_unet_destroy", "lbm_unet_param_count",
           "lbm_unet_set_params", "lbm_unet_get_params", "lbm_unet_forward", "lbm_unet_loss", "lbm_unet_backward",
           "lbm_unet_train_step", "lbm_unet_set_lr", "lbm_unet_save", "lbm_unet_load", "lbm_unet_encode",
           "lbm_unet_target", "lbm_unet_warm_rho", "lbm_unet_last_error")


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} not built: run `python -m paper_2202_06516_amd.build`")
    # PyTorch for ROCm ships its own HIP runtime under the same soname.  Loaded
    # first, it also serves this library and the process holds one runtime;
    # loaded after this library, it would bring a second runtime that then
    # finds no GPU.  So import it first when it is installed.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, vp, i, i64, d = C.POINTER, C.c_void_p, C.c_int, C.c_int64, C.c_double
    L.lbm_config_default.restype = None
    L.lbm_config_default.argtypes = [P(lbm_config), i]
    L.lbm_create.argtypes = [P(lbm_config), P(vp)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_set_solid.argtypes = [vp, P(lbm_solid), i, P(d)]
    L.lbm_init_drops.argtypes = [vp, P(lbm_drop), i, d]
    L.lbm_step.argtypes = [vp, i64, i, P(lbm_angle), i, P(i)]
    L.lbm_set_measure.argtypes = [vp, P(lbm_measure_opts)]
    L.lbm_measure_angle.argtypes = [vp, P(lbm_measure_opts), P(lbm_angle)]
    L.lbm_young_force.argtypes = [vp, P(lbm_young_opts), P(lbm_angle), P(lbm_young)]
    L.lbm_set_young.argtypes = [vp, P(lbm_young_opts)]
    L.lbm_young_series.argtypes = [vp, P(lbm_young), i, P(i)]
    L.lbm_read.argtypes = [vp, i, vp, C.c_size_t, i]
    L.lbm_write.argtypes = [vp, i, vp, C.c_size_t, i]
    L.lbm_sync.argtypes = [vp]
    L.lbm_get_info.argtypes = [vp, P(lbm_info)]
    L.lbm_profile_step.argtypes = [vp, i64, P(C.c_char_p), P(d), i, P(i)]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_last_error.argtypes = [vp]
    L.lbm_measure_field.argtypes = [i, i, P(i), vp, vp, P(lbm_solid), i, d, P(d), vp, vp]
    L.lbm_measure_field.restype = C.c_int
    L.lbm_batch_create.argtypes = [P(lbm_config), P(lbm_case), i, P(lbm_batch_opts), P(vp)]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_step.argtypes = [vp, i64, i]
    L.lbm_batch_sync.argtypes = [vp]
    L.lbm_batch_angles.argtypes = [vp, P(lbm_angle), i]
    L.lbm_batch_measure.argtypes = [vp, P(lbm_angle), i]
    L.lbm_batch_young_force.argtypes = [vp, P(lbm_young_opts), P(lbm_angle), P(lbm_young), i]
    L.lbm_batch_set_young.argtypes = [vp, P(lbm_young_opts)]
    L.lbm_batch_young_last.argtypes = [vp, P(lbm_young), i]
    L.lbm_batch_read.argtypes = [vp, i, i, vp, C.c_size_t, i]
    L.lbm_batch_write.argtypes = [vp, i, i, vp, C.c_size_t, i]
    L.lbm_batch_get_info.argtypes = [vp, P(lbm_batch_info)]
    L.lbm_batch_tune.argtypes = [vp, C.c_char_p]
    L.lbm_batch_profile_step.argtypes = [vp, i64, P(C.c_char_p), P(d), i, P(i)]
    L.lbm_batch_last_error.restype = C.c_char_p
    L.lbm_batch_last_error.argtypes = [vp]
    L.lbm_unet_config_default.restype = None
    L.lbm_unet_config_default.argtypes = [P(lbm_unet_config)]
    L.lbm_unet_create.argtypes = [P(lbm_unet_config), P(vp)]
    L.lbm_unet_destroy.argtypes = [vp]
    L.lbm_unet_param_count.restype = i64
    L.lbm_unet_param_count.argtypes = [vp]
    L.lbm_unet_set_params.argtypes = [vp, vp, i64, i]
    L.lbm_unet_get_params.argtypes = [vp, vp, i64, i, i]
    L.lbm_unet_forward.argtypes = [vp, vp, vp, i]
    L.lbm_unet_backward.argtypes = [vp, vp, vp, i, P(d)]
    L.lbm_unet_loss.argtypes = [vp, vp, vp, i, P(d)]
    L.lbm_unet_train_step.argtypes = [vp, vp, vp, i, P(d)]
    L.lbm_unet_set_lr.argtypes = [vp, d]
    L.lbm_unet_save.argtypes = [vp, C.c_char_p]
    L.lbm_unet_load.argtypes = [vp, C.c_char_p]
    L.lbm_unet_encode.argtypes = [vp, vp, i64, d, d, vp, vp]
    L.lbm_unet_target.argtypes = [vp, i, vp, i64, d, d, vp, vp]
    L.lbm_unet_warm_rho.argtypes = [vp, vp, vp, vp, i, i, i, d, d, d, i, vp, P(d)]
    L.lbm_unet_last_error.restype = C.c_char_p
    L.lbm_unet_last_error.argtypes = [vp]
    for name in ("lbm_unet_create", "lbm_unet_destroy", "lbm_unet_set_params", "lbm_unet_get_params",
                 "lbm_unet_forward", "lbm_unet_loss", "lbm_unet_backward", "lbm_unet_train_step", "lbm_unet_set_lr",
                 "lbm_unet_save", "lbm_unet_load",
                 "lbm_unet_encode", "lbm_unet_target", "lbm_unet_warm_rho"):
        getattr(L, name).restype = C.c_int
    for name in ("lbm_create", "lbm_destroy", "lbm_set_solid", "lbm_init_drops", "lbm_step",
                 "lbm_set_measure", "lbm_measure_angle", "lbm_read", "lbm_write", "lbm_sync",
                 "lbm_get_info", "lbm_profile_step", "lbm_young_force", "lbm_set_young", "lbm_young_series",
                 "lbm_batch_create", "lbm_batch_destroy",
                 "lbm_batch_step",
                 "lbm_batch_sync", "lbm_batch_angles", "lbm_batch_measure", "lbm_batch_young_force",
                 "lbm_batch_set_young", "lbm_batch_young_last",
                 "lbm_batch_read", "lbm_batch_write", "lbm_batch_get_info", "lbm_batch_tune", "lbm_batch_profile_step"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def measure_field(lattice, precision, n, rho_ptr, cls_ptr, solid, n_sectors, rho_m, out_ptr, g=None, stream=None):
    """lbm_measure_field: the contact angle of a device density field into the device buffer at out_ptr
    (one lbm_angle); enqueues on stream and returns without synchronising."""
    nn = (C.c_int * 3)(*(list(n) + [1] * (3 - len(n))))
    sd = lbm_solid()
    _fill_solid(sd, solid)
    gg = None
    if g is not None:
        gg = (C.c_double * 3)(*(list(g) + [0.0] * (3 - len(g))))
    st = lib().lbm_measure_field(int(lattice), int(precision), nn, C.c_void_p(rho_ptr), C.c_void_p(cls_ptr),
                                 C.byref(sd), int(n_sectors), float(rho_m), gg, C.c_void_p(out_ptr),
                                 C.c_void_p(stream) if stream else None)
    if st != 0:
        raise LbmError(st, lib().lbm_last_error(None).decode())


def config_default(lattice: int) -> lbm_config:
    cfg = lbm_config()
    lib().lbm_config_default(C.byref(cfg), lattice)
    return cfg


class Lattice:
    """One lbm context: create, set solids, initialise, step, measure, read."""

    def __init__(self, lattice=LBM_D2Q9, n=(128, 128, 1), precision=None, axis_bc=(0, 0, 0), stream=None,
                 **params):
        cfg = config_default(lattice)
        if precision is not None:
            cfg.precision = precision
        nn = list(n) + [1] * (3 - len(n))
        for k in range(3):
            cfg.n[k] = nn[k]
            cfg.axis_bc[k] = axis_bc[k] if k < len(axis_bc) else 0
        for key, val in params.items():
            if key == "g":
                for k in range(3):
                    cfg.g[k] = val[k] if k < len(val) else 0.0
            else:
                if not hasattr(cfg, key):
                    raise KeyError(key)
                setattr(cfg, key, val)
        if stream is not None:
            cfg.stream = stream
        self.cfg = cfg
        self.dim = 2 if lattice == LBM_D2Q9 else 3
        self.Q = 9 if self.dim == 2 else 19
        self.shape = (1 if self.dim == 2 else nn[2], nn[1], nn[0])
        self.N = int(np.prod(self.shape))
        self.dtype = np.float64 if cfg.precision == LBM_F64 else np.float32
        h = C.c_void_p()
        st = lib().lbm_create(C.byref(cfg), C.byref(h))
        if st != 0:
            raise LbmError(st, "lbm_create failed (invalid configuration?)")
        self._h = h

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: module globals may be gone
            pass

    def _check(self, st):
        if st != 0:
            raise LbmError(st, lib().lbm_last_error(self._h).decode())
        return st

    # -- set-up ------------------------------------------------------------
    def set_solids(self, solids, mu_w_map=None):
        """solids: dicts with center, radius, mu_w or stripes=(mu_w, mu_w2, width),
        optional pole, and cavity=True for the concave substrate (solid outside)."""
        arr = (lbm_solid * max(len(solids), 1))()
        for i, s in enumerate(solids):
            _fill_solid(arr[i], s)
        mp = None
        if mu_w_map is not None:
            self._muw = np.ascontiguousarray(mu_w_map, dtype=np.float64).reshape(-1)
            mp = self._muw.ctypes.data_as(C.POINTER(C.c_double))
        self._check(lib().lbm_set_solid(self._h, arr, len(solids), mp))

    def init_drops(self, drops, W=10.0):
        arr = (lbm_drop * len(drops))()
        for i, (c, r) in enumerate(drops):
            cc = list(c) + [0.0] * (3 - len(c))
            for k in range(3):
                arr[i].center[k] = cc[k]
            arr[i].radius = r
        self._check(lib().lbm_init_drops(self._h, arr, len(drops), float(W)))

    def set_measure(self, solid_index=0, n_sectors=32, rho_m=0.0):
        o = lbm_measure_opts(solid_index, n_sectors, rho_m)
        self._check(lib().lbm_set_measure(self._h, C.byref(o)))

    # -- stepping ----------------------------------------------------------
    def step(self, n, measure_every=0, cap=0):
        if cap:
            arr = (lbm_angle * cap)()
            nw = C.c_int()
            self._check(lib().lbm_step(self._h, int(n), int(measure_every), arr, cap, C.byref(nw)))
            self._series_len = nw.value
            return [arr[i] for i in range(nw.value)]
        self._check(lib().lbm_step(self._h, int(n), int(measure_every), None, 0, None))
        self._series_len = 0
        return []

    def sync(self):
        self._check(lib().lbm_sync(self._h))

    def measure(self, solid_index=0, n_sectors=32, rho_m=0.0, allow_missing=True):
        o = lbm_measure_opts(solid_index, n_sectors, rho_m)
        a = lbm_angle()
        st = lib().lbm_measure_angle(self._h, C.byref(o), C.byref(a))
        if st not in (0, LBM_E_NO_CONTACT_LINE) or (st != 0 and not allow_missing):
            self._check(st)
        return a

    def young_force(self, gamma, theta1_deg, theta2_deg=90.0, roughness=1.0, band=(0.1, 0.9)):
        """Measure now (lbm_set_measure's options) and return (lbm_angle, lbm_young): Eq. 17 and Eq. 18
        per sector; NaN values and status LBM_E_NO_CONTACT_LINE when there is no contact line."""
        o = lbm_young_opts(float(gamma), float(theta1_deg), float(theta2_deg), float(roughness), float(band[0]),
                           float(band[1]))
        a, y = lbm_angle(), lbm_young()
        st = lib().lbm_young_force(self._h, C.byref(o), C.byref(a), C.byref(y))
        if st not in (0, LBM_E_NO_CONTACT_LINE):
            self._check(st)
        return a, y

    def set_young(self, gamma=None, theta1_deg=90.0, theta2_deg=90.0, roughness=1.0, band=(0.1, 0.9)):
        """Take the unbalanced Young force at every in-step measurement (gamma None: off)."""
        if gamma is None:
            self._check(lib().lbm_set_young(self._h, None))
            return
        o = lbm_young_opts(float(gamma), float(theta1_deg), float(theta2_deg), float(roughness), float(band[0]),
                           float(band[1]))
        self._check(lib().lbm_set_young(self._h, C.byref(o)))

    def young_series(self, cap=None):
        """Young-force records of the last step call that wrote an angle series (all of them unless cap is
        given)."""
        if cap is None:
            cap = getattr(self, "_series_len", 0)
        arr = (lbm_young * max(cap, 1))()
        n = C.c_int()
        self._check(lib().lbm_young_series(self._h, arr, cap, C.byref(n)))
        return [arr[k] for k in range(n.value)]

    # -- fields ------------------------------------------------------------
    def read(self, field):
        if field == FIELD_CLASS:
            out = np.empty(self.shape, dtype=np.uint8)
        elif field == FIELD_MASS:
            out = np.empty(1, dtype=np.float64)
        elif field in (FIELD_F, FIELD_G):
            out = np.empty((self.Q,) + self.shape, dtype=self.dtype)
        elif field == FIELD_VEL:
            out = np.empty((3,) + self.shape, dtype=self.dtype)
        else:
            out = np.empty(self.shape, dtype=self.dtype)
        self._check(lib().lbm_read(self._h, field, out.ctypes.data, out.nbytes, 0))
        return out[0] if field == FIELD_MASS else out

    def read_device(self, field, ptr, nbytes):
        self._check(lib().lbm_read(self._h, field, C.c_void_p(ptr), nbytes, 1))

    def write(self, field, arr):
        a = np.ascontiguousarray(arr, dtype=self.dtype)
        self._check(lib().lbm_write(self._h, field, a.ctypes.data, a.nbytes, 0))

    def write_device(self, field, ptr, nbytes):
        """Replace RHO (then f = f_eq(rho, 0)) or F from device memory at ptr."""
        self._check(lib().lbm_write(self._h, field, C.c_void_p(ptr), nbytes, 1))

    @property
    def rho(self):
        return self.read(FIELD_RHO)

    @property
    def f(self):
        return self.read(FIELD_F)

    @property
    def phi(self):
        """Order parameter of the phase-field model."""
        return self.read(FIELD_PHI)

    @property
    def g(self):
        """Order-parameter populations S_t of the phase-field model."""
        return self.read(FIELD_G)

    def mass(self):
        return float(self.read(FIELD_MASS))

    def info(self):
        inf = lbm_info()
        self._check(lib().lbm_get_info(self._h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in lbm_info._fields_}

    def profile(self, nsteps):
        names = (C.c_char_p * 8)()
        ms = (C.c_double * 8)()
        n = C.c_int()
        self._check(lib().lbm_profile_step(self._h, int(nsteps), names, ms, 8, C.byref(n)))
        return {names[i].decode(): ms[i] for i in range(n.value)}


def _fill_solid(dst, s):
    dst.kind = LBM_SOLID_CAVITY if s.get("cavity") else LBM_SOLID_SPHERE
    c = list(s["center"]) + [0.0] * (3 - len(s["center"]))
    for k in range(3):
        dst.center[k] = c[k]
    dst.radius = s["radius"]
    if "stripes" in s:
        dst.wet_mode = LBM_WET_STRIPES
        dst.mu_w, dst.mu_w2, dst.stripe_width = s["stripes"]
    else:
        dst.wet_mode = LBM_WET_UNIFORM
        dst.mu_w = s.get("mu_w", 0.0)
    pole = s.get("pole", (0.0, 0.0, 0.0))
    for k in range(3):
        dst.pole[k] = pole[k] if k < len(pole) else 0.0


class Batch:
    """Many independent lattices (one solid and one drop each) advanced together."""

    def __init__(self, cases, lattice=LBM_D2Q9, precision=LBM_F32, axis_bc=(0, 0, 0), autotune=False, tile_w=64,
                 blocks_per_cu=4, cache_path=None, stream=None, **params):
        cfg = config_default(lattice)
        cfg.precision = precision
        for k in range(3):
            cfg.axis_bc[k] = axis_bc[k] if k < len(axis_bc) else 0
        for key, val in params.items():
            if key == "g":
                for k in range(3):
                    cfg.g[k] = val[k] if k < len(val) else 0.0
            else:
                if not hasattr(cfg, key):
                    raise KeyError(key)
                setattr(cfg, key, val)
        if stream is not None:
            cfg.stream = stream
        self.cfg = cfg
        self.dim = 2 if lattice == LBM_D2Q9 else 3
        self.Q = 9 if self.dim == 2 else 19
        self.dtype = np.float64 if precision == LBM_F64 else np.float32
        arr = (lbm_case * len(cases))()
        self.shapes = []
        for i, cs in enumerate(cases):
            n = list(cs["n"]) + [1] * (3 - len(cs["n"]))
            for k in range(3):
                arr[i].n[k] = n[k]
            _fill_solid(arr[i].solid, cs["solid"])
            c, r = cs["drop"]
            cc = list(c) + [0.0] * (3 - len(c))
            for k in range(3):
                arr[i].drop.center[k] = cc[k]
            arr[i].drop.radius = r
            self.shapes.append((n[2], n[1], n[0]))
        self._cache = cache_path.encode() if cache_path else None
        opts = lbm_batch_opts(int(autotune), tile_w, blocks_per_cu, self._cache)
        h = C.c_void_p()
        st = lib().lbm_batch_create(C.byref(cfg), arr, len(cases), C.byref(opts), C.byref(h))
        if st != 0:
            raise LbmError(st, "lbm_batch_create failed")
        self._h = h
        self.ncases = len(cases)

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: module globals may be gone
            pass

    def _check(self, st):
        if st != 0:
            raise LbmError(st, lib().lbm_batch_last_error(self._h).decode())

    def step(self, n, measure_every=0):
        self._check(lib().lbm_batch_step(self._h, int(n), int(measure_every)))

    def sync(self):
        self._check(lib().lbm_batch_sync(self._h))

    def angles(self):
        arr = (lbm_angle * self.ncases)()
        self._check(lib().lbm_batch_angles(self._h, arr, self.ncases))
        return list(arr)

    def measure(self):
        arr = (lbm_angle * self.ncases)()
        self._check(lib().lbm_batch_measure(self._h, arr, self.ncases))
        return list(arr)

    def set_young(self, gamma=None, theta1_deg=90.0, theta2_deg=90.0, roughness=1.0, band=(0.1, 0.9)):
        """Take the unbalanced Young force at every in-step measurement of every case (gamma None: off)."""
        if gamma is None:
            self._check(lib().lbm_batch_set_young(self._h, None))
            return
        o = lbm_young_opts(float(gamma), float(theta1_deg), float(theta2_deg), float(roughness), float(band[0]),
                           float(band[1]))
        self._check(lib().lbm_batch_set_young(self._h, C.byref(o)))

    def young_last(self):
        """The latest in-step Young-force record of every case."""
        arr = (lbm_young * self.ncases)()
        self._check(lib().lbm_batch_young_last(self._h, arr, self.ncases))
        return list(arr)

    def young_force(self, gamma, theta1_deg, theta2_deg=90.0, roughness=1.0, band=(0.1, 0.9)):
        """Measure every case now and return (angles, youngs): Eq. 17 and Eq. 18 per case and sector; a case
        without a contact line has status LBM_E_NO_CONTACT_LINE and NaN values."""
        o = lbm_young_opts(float(gamma), float(theta1_deg), float(theta2_deg), float(roughness), float(band[0]),
                           float(band[1]))
        a, y = (lbm_angle * self.ncases)(), (lbm_young * self.ncases)()
        self._check(lib().lbm_batch_young_force(self._h, C.byref(o), a, y, self.ncases))
        return list(a), list(y)

    def read(self, case, field):
        shp = self.shapes[case]
        if field == FIELD_CLASS:
            out = np.empty(shp, dtype=np.uint8)
        elif field in (FIELD_F, FIELD_G):
            out = np.empty((self.Q,) + shp, dtype=self.dtype)
        else:
            out = np.empty(shp, dtype=self.dtype)
        self._check(lib().lbm_batch_read(self._h, case, field, out.ctypes.data, out.nbytes, 0))
        return out

    def write_rho(self, case, rho):
        a = np.ascontiguousarray(rho, dtype=self.dtype)
        self._check(lib().lbm_batch_write(self._h, case, FIELD_RHO, a.ctypes.data, a.nbytes, 0))

    def write_phi(self, case, phi):
        """Phase-field model: the state at rest of an order-parameter field for one case."""
        a = np.ascontiguousarray(phi, dtype=self.dtype)
        self._check(lib().lbm_batch_write(self._h, case, FIELD_PHI, a.ctypes.data, a.nbytes, 0))

    def read_device(self, case, field, ptr, nbytes):
        """Copy one case's field into device memory at ptr."""
        self._check(lib().lbm_batch_read(self._h, case, field, C.c_void_p(ptr), nbytes, 1))

    def write_rho_device(self, case, ptr, nbytes):
        self._check(lib().lbm_batch_write(self._h, case, FIELD_RHO, C.c_void_p(ptr), nbytes, 1))

    def info(self):
        inf = lbm_batch_info()
        self._check(lib().lbm_batch_get_info(self._h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in lbm_batch_info._fields_}

    def tune(self, cache_path=None):
        self._check(lib().lbm_batch_tune(self._h, cache_path.encode() if cache_path else None))

    def profile(self, nsteps):
        """Mean ms per launch of kb_density, kb_mu and kb_collide over nsteps eager steps."""
        names = (C.c_char_p * 8)()
        ms = (C.c_double * 8)()
        n = C.c_int()
        self._check(lib().lbm_batch_profile_step(self._h, int(nsteps), names, ms, 8, C.byref(n)))
        return {names[i].decode(): ms[i] for i in range(n.value)}


class Unet:
    """The warm-start U-Net (lbm_unet_*): device pointers in, device pointers out.

    Arrays are passed as integer device addresses (for instance
    ``tensor.data_ptr()`` of a contiguous torch tensor on the GPU) or, for
    parameters, as host numpy arrays.
    """

    def __init__(self, H=256, W=256, batch=8, in_channels=3, base_channels=32, levels=4, lr=1e-3,
                 beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        cfg = lbm_unet_config()
        lib().lbm_unet_config_default(C.byref(cfg))
        cfg.H, cfg.W, cfg.batch, cfg.in_channels = H, W, batch, in_channels
        cfg.base_channels, cfg.levels = base_channels, levels
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = lr, beta1, beta2, eps
        if stream is not None:
            cfg.stream = stream
        self.cfg = cfg
        h = C.c_void_p()
        st = lib().lbm_unet_create(C.byref(cfg), C.byref(h))
        if st != 0:
            raise LbmError(st, "lbm_unet_create failed")
        self._h = h
        self.n_params = int(lib().lbm_unet_param_count(h))

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: module globals may be gone
            pass

    def _check(self, st):
        if st != 0:
            raise LbmError(st, lib().lbm_unet_last_error(self._h).decode())

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
        self._check(lib().lbm_unet_set_params(self._h, a.ctypes.data, a.size, 0))

    def params(self, which=LBM_UNET_WEIGHTS):
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(lib().lbm_unet_get_params(self._h, out.ctypes.data, out.size, which, 0))
        return out

    def grads(self):
        return self.params(LBM_UNET_GRADS)

    def forward(self, x_ptr, y_ptr, n):
        self._check(lib().lbm_unet_forward(self._h, C.c_void_p(x_ptr), C.c_void_p(y_ptr), int(n)))

    def loss(self, x_ptr, t_ptr, n):
        loss = C.c_double()
        self._check(lib().lbm_unet_loss(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), int(n), C.byref(loss)))
        return loss.value

    def backward(self, x_ptr, t_ptr, n):
        loss = C.c_double()
        self._check(lib().lbm_unet_backward(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), int(n), C.byref(loss)))
        return loss.value

    def train_step(self, x_ptr, t_ptr, n):
        loss = C.c_double()
        self._check(lib().lbm_unet_train_step(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), int(n),
                                              C.byref(loss)))
        return loss.value

    def set_lr(self, lr):
        self._check(lib().lbm_unet_set_lr(self._h, float(lr)))

    def save(self, path):
        self._check(lib().lbm_unet_save(self._h, str(path).encode()))

    def load(self, path):
        self._check(lib().lbm_unet_load(self._h, str(path).encode()))

    def warm_rho(self, phi_ptr, rho_ref_ptr, cls_ptr, nx, ny, precision, rho_g, rho_l, rho_out_ptr, cut=0.0,
                 smooth=0):
        info = (C.c_double * 5)()
        self._check(lib().lbm_unet_warm_rho(self._h, C.c_void_p(phi_ptr), C.c_void_p(rho_ref_ptr),
                                            C.c_void_p(cls_ptr), int(nx), int(ny), int(precision), float(rho_g),
                                            float(rho_l), float(cut), int(smooth), C.c_void_p(rho_out_ptr), info))
        return dict(mass_ref=info[0], mass_written=info[1], delta=info[2], scale=info[3], n_fluid=info[4])


def unet_encode(cls_ptr, n, solid_value, plane, x_ptr, stream=None, phi0_ptr=None):
    st = lib().lbm_unet_encode(C.c_void_p(cls_ptr), C.c_void_p(phi0_ptr) if phi0_ptr else None, int(n),
                               float(solid_value), float(plane), C.c_void_p(x_ptr),
                               C.c_void_p(stream) if stream else None)
    if st != 0:
        raise LbmError(st, "lbm_unet_encode failed")


def unet_target(rho_ptr, precision, cls_ptr, n, rho_g, rho_l, phi_ptr, stream=None):
    st = lib().lbm_unet_target(C.c_void_p(rho_ptr), int(precision), C.c_void_p(cls_ptr), int(n), float(rho_g),
                               float(rho_l), C.c_void_p(phi_ptr), C.c_void_p(stream) if stream else None)
    if st != 0:
        raise LbmError(st, "lbm_unet_target failed")


def angle_dict(a):
    return dict(step=a.step, status=a.status, mean=a.mean_deg, adv=a.adv_deg, rec=a.rec_deg,
                sectors=list(a.sector_deg[: a.n_sectors]), n_valid=a.n_valid)


__all__ = [n for n in dir() if not n.startswith("_")] + ["math"]
