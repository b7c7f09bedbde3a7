"""FP64 CPU oracle for the multiphase lattice Boltzmann step of arXiv:2202.06516.

TEST INFRASTRUCTURE ONLY.  This package is the correctness oracle: the tests,
the smoke check and the benchmark's CPU-baseline leg load it, and nothing in
the product path does.  It shares no code with the GPU library.

The arithmetic lives in ``lbm_oracle.c`` (plain loops, double precision, no
FMA contraction); this module only marshals arguments with ctypes and exposes
the fields as numpy views.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int * 3), ("wall", C.c_int * 3), ("bgk", C.c_int),
        ("bc_mode", C.c_int),
        ("tau", C.c_double), ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
        ("s_pi", C.c_double), ("s_m", C.c_double),
        ("Tr", C.c_double), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
        ("omega", C.c_double), ("k", C.c_double), ("kappa", C.c_double),
        ("g", C.c_double * 3), ("g_start", C.c_longlong),
        ("rho_l", C.c_double), ("rho_g", C.c_double), ("wall_mu", C.c_double),
        ("model", C.c_int), ("sc_G", C.c_double),
        ("pf_A", C.c_double), ("pf_kappa", C.c_double), ("pf_gamma", C.c_double), ("pf_tau", C.c_double),
        ("pf_rho0", C.c_double),
    ]


class Angle(C.Structure):
    _fields_ = [
        ("step", C.c_longlong), ("status", C.c_int), ("n_sectors", C.c_int), ("n_valid", C.c_int),
        ("mean_deg", C.c_double), ("adv_deg", C.c_double), ("rec_deg", C.c_double),
        ("axis", C.c_double * 3), ("sector_deg", C.c_double * 64),
        ("contact", (C.c_double * 3) * 64), ("p1", (C.c_double * 3) * 64), ("p2", (C.c_double * 3) * 64),
        ("key1", C.c_ulonglong * 64), ("key2", C.c_ulonglong * 64),
    ]

    def sectors(self):
        return np.array(self.sector_deg[: self.n_sectors])


class Young(C.Structure):
    _fields_ = [
        ("step", C.c_longlong), ("status", C.c_int), ("n_sectors", C.c_int),
        ("count", (C.c_int * 2) * 64), ("phi_d", C.c_double * 64), ("theta_eq_deg", C.c_double * 64),
        ("force", C.c_double * 64),
    ]


_lib = None


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's loops from now on (same libgomp instance as
    the oracle library); returns the number in effect."""
    lib()
    g = C.CDLL("libgomp.so.1")
    g.omp_set_num_threads(C.c_int(int(n)))
    g.omp_get_max_threads.restype = C.c_int
    return int(g.omp_get_max_threads())


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        d, i, v, p = C.c_double, C.c_int, C.c_void_p, C.POINTER
        L.ora_pr_alpha.restype = d; L.ora_pr_alpha.argtypes = [d, d]
        L.ora_pr_p0.restype = d; L.ora_pr_p0.argtypes = [d] * 6
        L.ora_pr_mu.restype = d; L.ora_pr_mu.argtypes = [d] * 6
        L.ora_pr_critical.argtypes = [d, d, d, p(d), p(d), p(d)]
        L.ora_maxwell.argtypes = [d, d, d, d, d, p(d), p(d), p(d), p(d)]
        L.ora_lattice.argtypes = [i, p(i), p(i), p(d)]
        L.ora_mrt_matrix.argtypes = [i, p(d)]
        L.ora_feq.argtypes = [i, d, p(d), p(d)]
        L.ora_collide_node.argtypes = [p(Params), p(d), p(d), p(d)]
        L.ora_create.restype = v; L.ora_create.argtypes = [p(Params)]
        L.ora_destroy.argtypes = [v]
        L.ora_add_sphere.argtypes = [v, p(d), d, i, d, d, d, p(d)]
        L.ora_add_cavity.argtypes = [v, p(d), d, i, d, d, d, p(d)]
        L.ora_set_muw_map.argtypes = [v, p(d)]
        L.ora_build.argtypes = [v]
        L.ora_init_drops.argtypes = [v, p(d), p(d), i, d]
        L.ora_set_rho.argtypes = [v, p(d)]
        L.ora_step.argtypes = [v, C.c_longlong]
        L.ora_step_measured.argtypes = [v, C.c_longlong, i, i, i, d, p(Angle), i, p(i)]
        L.ora_measure.argtypes = [v, i, i, d, p(Angle)]
        L.ora_young_force.argtypes = [v, i, i, d, d, d, d, d, d, d, p(Angle), p(Young)]
        L.ora_field.restype = v; L.ora_field.argtypes = [v, i]
        L.ora_update_derived.argtypes = [v]
        L.ora_velocity.argtypes = [v, p(d)]
        L.ora_mass.restype = d; L.ora_mass.argtypes = [v]
        L.ora_get_step.restype = C.c_longlong; L.ora_get_step.argtypes = [v]
        L.ora_get_info.argtypes = [v, p(d)]
        for ph in ("density", "fill", "mu", "force", "collide", "stream"):
            getattr(L, "ora_phase_" + ph).argtypes = [v]
        L.ora_link_q.restype = d; L.ora_link_q.argtypes = [v, i, i, i, i]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# --------------------------------------------------------------------------
# thermodynamics
# --------------------------------------------------------------------------
PR_A, PR_B, PR_R, PR_OMEGA = 2.0 / 49.0, 2.0 / 21.0, 1.0, 0.344


def pr_alpha(Tr, omega=PR_OMEGA):
    return lib().ora_pr_alpha(Tr, omega)


def pr_critical(a=PR_A, b=PR_B, R=PR_R):
    Tc, rc, pc = C.c_double(), C.c_double(), C.c_double()
    lib().ora_pr_critical(a, b, R, C.byref(Tc), C.byref(rc), C.byref(pc))
    return Tc.value, rc.value, pc.value


def pr_p0(rho, T, alpha, a=PR_A, b=PR_B, R=PR_R):
    return lib().ora_pr_p0(rho, T, a, b, R, alpha)


def pr_mu(rho, T, alpha, a=PR_A, b=PR_B, R=PR_R):
    return lib().ora_pr_mu(rho, T, a, b, R, alpha)


def maxwell(Tr, a=PR_A, b=PR_B, R=PR_R, omega=PR_OMEGA):
    Tc = pr_critical(a, b, R)[0]
    T = Tr * Tc
    al = pr_alpha(Tr, omega)
    rg, rl, ps, ms = (C.c_double() for _ in range(4))
    rc = lib().ora_maxwell(T, a, b, R, al, C.byref(rg), C.byref(rl), C.byref(ps), C.byref(ms))
    if rc != 0:
        raise RuntimeError("Maxwell construction failed")
    return dict(T=T, Tc=Tc, alpha=al, rho_g=rg.value, rho_l=rl.value, p_sat=ps.value, mu_sat=ms.value)


def lattice(dim):
    Q = C.c_int()
    e = np.zeros(19 * 3, dtype=np.int32)
    w = np.zeros(19)
    lib().ora_lattice(dim, C.byref(Q), e.ctypes.data_as(C.POINTER(C.c_int)), _dp(w))
    q = Q.value
    return e[: 3 * q].reshape(q, 3).copy(), w[:q].copy()


def mrt_matrix(dim):
    q = 9 if dim == 2 else 19
    M = np.zeros(q * q)
    lib().ora_mrt_matrix(dim, _dp(M))
    return M.reshape(q, q)


def feq(dim, rho, u):
    q = 9 if dim == 2 else 19
    out = np.zeros(q)
    uu = np.zeros(3)
    uu[: len(u)] = u
    lib().ora_feq(dim, rho, _dp(uu), _dp(out))
    return out


# --------------------------------------------------------------------------
# simulation context
# --------------------------------------------------------------------------
DEFAULTS = dict(tau=1.0, s_e=1.64, s_eps=1.54, s_q=1.9, s_pi=1.54, s_m=1.9,
                Tr=0.6, a=PR_A, b=PR_B, R=PR_R, omega=PR_OMEGA, k=0.28, kappa=0.01,
                g=(0.0, 0.0, 0.0), g_start=0, rho_l=0.0, rho_g=0.0, wall_mu=math.nan,
                bgk=0, bc_mode=0, model=0, sc_G=0.0,
                pf_A=0.01, pf_kappa=0.02, pf_gamma=1.0, pf_tau=1.0, pf_rho0=1.0)


def make_params(dim, n, wall=(0, 0, 0), **kw):
    cfg = dict(DEFAULTS)
    cfg.update(kw)
    p = Params()
    p.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    for d in range(3):
        p.n[d] = nn[d]
        p.wall[d] = int(wall[d]) if d < len(wall) else 0
        p.g[d] = cfg["g"][d] if d < len(cfg["g"]) else 0.0
    for name in ("bgk", "bc_mode"):
        setattr(p, name, int(cfg[name]))
    for name in ("tau", "s_e", "s_eps", "s_q", "s_pi", "s_m", "Tr", "a", "b", "R", "omega",
                 "k", "kappa", "rho_l", "rho_g", "wall_mu"):
        setattr(p, name, float(cfg[name]))
    p.g_start = int(cfg["g_start"])
    p.model = int(cfg["model"])
    p.sc_G = float(cfg["sc_G"])
    for name in ("pf_A", "pf_kappa", "pf_gamma", "pf_tau", "pf_rho0"):
        setattr(p, name, float(cfg[name]))
    return p


class Oracle:
    """A lattice, its solids and its populations, stepped on the CPU in FP64."""

    def __init__(self, dim, n, wall=(0, 0, 0), **kw):
        self.params = make_params(dim, n, wall, **kw)
        self.dim = dim
        self.Q = 9 if dim == 2 else 19
        self.shape = (1 if dim == 2 else n[2], n[1], n[0])
        self.N = int(np.prod(self.shape))
        self._h = lib().ora_create(C.byref(self.params))
        if not self._h:
            raise RuntimeError("ora_create failed")

    def close(self):
        if self._h:
            lib().ora_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def add_sphere(self, centre, radius, mu_w=0.0, stripes=None, pole=None, cavity=False):
        """Convex circle/ball (Fig. 2a), or with cavity=True the concave
        substrate of Fig. 2b: solid outside the circle/ball."""
        c = np.zeros(3)
        c[: len(centre)] = centre
        if stripes is None:
            mode, mu2, width = 0, 0.0, 1.0
        else:
            mode, (mu_w, mu2, width) = 1, stripes
        pl = None if pole is None else _dp(np.asarray(pole, dtype=np.float64))
        add = lib().ora_add_cavity if cavity else lib().ora_add_sphere
        rc = add(self._h, _dp(c), float(radius), mode, float(mu_w), float(mu2), float(width), pl)
        if rc != 0:
            raise ValueError("bad solid")
        lib().ora_build(self._h)

    def set_muw_map(self, m):
        self._muw = None if m is None else np.ascontiguousarray(m, dtype=np.float64).reshape(-1)
        lib().ora_set_muw_map(self._h, None if m is None else _dp(self._muw))

    def init_drops(self, centres, radii, W=10.0):
        cs = np.zeros((len(centres), 3))
        for i, c in enumerate(centres):
            cs[i, : len(c)] = c
        r = np.asarray(radii, dtype=np.float64)
        lib().ora_init_drops(self._h, _dp(cs), _dp(r), len(r), float(W))

    def set_rho(self, rho):
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        lib().ora_set_rho(self._h, _dp(r))

    def step(self, n):
        lib().ora_step(self._h, int(n))

    def step_measured(self, n, every, solid=0, n_sectors=2, rho_m=0.0, cap=None):
        cap = cap or (int(n) // max(every, 1) + 2)
        arr = (Angle * cap)()
        nw = C.c_int()
        lib().ora_step_measured(self._h, int(n), int(every), solid, n_sectors, rho_m, arr, cap, C.byref(nw))
        return [arr[i] for i in range(nw.value)]

    def measure(self, solid=0, n_sectors=2, rho_m=0.0):
        a = Angle()
        lib().ora_measure(self._h, solid, n_sectors, float(rho_m), C.byref(a))
        return a

    def young_force(self, gamma, theta1_deg, theta2_deg, roughness=1.0, band=(0.1, 0.9), solid=0, n_sectors=2,
                    rho_m=0.0):
        """Eq. 17 / Eq. 18 per sector on a measurement made now: (Angle, Young)."""
        a, y = Angle(), Young()
        lib().ora_young_force(self._h, solid, n_sectors, float(rho_m), float(band[0]), float(band[1]), float(gamma),
                              float(theta1_deg), float(theta2_deg), float(roughness), C.byref(a), C.byref(y))
        return a, y

    def _view(self, which, count, dtype=np.float64):
        ptr = lib().ora_field(self._h, which)
        ct = C.c_double if dtype == np.float64 else C.c_ubyte
        buf = (ct * count).from_address(ptr)
        return np.frombuffer(buf, dtype=dtype, count=count)

    @property
    def f(self):
        return self._view(0, self.Q * self.N).reshape((self.Q,) + self.shape)

    @property
    def fpost(self):
        return self._view(5, self.Q * self.N).reshape((self.Q,) + self.shape)

    @property
    def rho(self):
        return self._view(1, self.N).reshape(self.shape)

    @property
    def phi(self):
        """Order parameter of the phase-field model."""
        return self._view(6, self.N).reshape(self.shape)

    @property
    def g(self):
        """Order-parameter populations of the phase-field model (state)."""
        return self._view(7, self.Q * self.N).reshape((self.Q,) + self.shape)

    @property
    def mu(self):
        return self._view(2, self.N).reshape(self.shape)

    @property
    def force(self):
        return self._view(3, 3 * self.N).reshape((3,) + self.shape)

    @property
    def cls(self):
        return self._view(4, self.N, np.uint8).reshape(self.shape)

    def update_derived(self):
        lib().ora_update_derived(self._h)

    def phase(self, name):
        getattr(lib(), "ora_phase_" + name)(self._h)

    def velocity(self):
        v = np.zeros(3 * self.N)
        lib().ora_velocity(self._h, _dp(v))
        return v.reshape((3,) + self.shape)

    def mass(self):
        return lib().ora_mass(self._h)

    @property
    def t(self):
        return lib().ora_get_step(self._h)

    def info(self):
        out = np.zeros(8)
        lib().ora_get_info(self._h, _dp(out))
        keys = ("Tc", "T", "alpha", "rho_g", "rho_l", "mu_sat", "p_sat", "wall_mu")
        return dict(zip(keys, out.tolist()))

    def link_q(self, x, y, z, d):
        return lib().ora_link_q(self._h, x, y, z, d)


def collide_node(params, f, F):
    f = np.ascontiguousarray(f, dtype=np.float64)
    FF = np.zeros(3)
    FF[: len(F)] = F
    out = np.zeros_like(f)
    lib().ora_collide_node(C.byref(params), _dp(f), _dp(FF), _dp(out))
    return out
