"""ctypes wrapper of the FP64 C oracle (test infrastructure only).

The parameter names are the paper's symbols (see lbm_oracle.c); the wrapper
only marshals numpy arrays and a parameter dict into C.
"""
import ctypes
import os

import numpy as np

from . import build as _build

Q19 = 19
Q7 = 7

_PARAM_FIELDS = [
    ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("bc_z", ctypes.c_int),
    ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
    ("acentric", ctypes.c_double), ("G", ctypes.c_double), ("sigma", ctypes.c_double),
    ("tau_e", ctypes.c_double), ("tau_v", ctypes.c_double), ("tau_q", ctypes.c_double),
    ("tau_pi", ctypes.c_double), ("cV", ctypes.c_double), ("d", ctypes.c_double),
    ("kappa_mode", ctypes.c_int), ("kappa", ctypes.c_double),
    ("vs_q", ctypes.c_double), ("vs_pi", ctypes.c_double), ("grav", ctypes.c_double * 3),
    ("T_wall_patch", ctypes.c_double), ("T_wall", ctypes.c_double),
    ("patch_radius", ctypes.c_double), ("T_top", ctypes.c_double), ("thermal", ctypes.c_int),
    ("bc_T_shell", ctypes.c_int), ("T_shell", ctypes.c_double), ("thermal_bgk", ctypes.c_int),
    ("thermal_lattice", ctypes.c_int), ("divu_mode", ctypes.c_int), ("freeze_flow", ctypes.c_int),
]


class OrcParams(ctypes.Structure):
    _fields_ = _PARAM_FIELDS


# Defaults follow Sec. IV: G = -1, acentric factor 0.344, d = 0.95, c_V = 5,
# tau_v = 0.8 (nu = 0.1), tau_e = 1.25, all other relaxation times 1.
DEFAULTS = dict(nx=8, ny=8, nz=8, bc_z=0, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, acentric=0.344,
                G=-1.0, sigma=0.0, tau_e=1.25, tau_v=0.8, tau_q=1.0, tau_pi=1.0, cV=5.0, d=0.95,
                kappa_mode=0, kappa=0.2, vs_q=1.0, vs_pi=1.0, grav=(0.0, 0.0, 0.0),
                T_wall_patch=0.0, T_wall=0.0, patch_radius=0.0, T_top=0.0, thermal=1, bc_T_shell=0, T_shell=0.0,
                thermal_bgk=0, thermal_lattice=0, divu_mode=0, freeze_flow=0)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(OrcParams)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        L.orc_create.argtypes = [P, ctypes.POINTER(vp)]
        L.orc_create.restype = ctypes.c_int
        L.orc_destroy.argtypes = [vp]
        L.orc_init_fields.argtypes = [vp, dp, dp, dp, dp, dp]
        L.orc_init_fields.restype = ctypes.c_int
        L.orc_step.argtypes = [vp, ctypes.c_int]
        L.orc_step.restype = ctypes.c_int
        L.orc_get_rho_u_T.argtypes = [vp, dp, dp, dp, dp, dp]
        L.orc_get_rho_u_T.restype = ctypes.c_int
        L.orc_get_state.argtypes = [vp, dp, dp, dp, dp]
        L.orc_set_state.argtypes = [vp, dp, dp, dp, ctypes.c_double]
        L.orc_reduce.argtypes = [vp, dp, dp]
        L.orc_tables.argtypes = [P, dp, dp, dp, dp, ip, ip, dp, dp]
        L.orc_critical_temperature.argtypes = [P]
        L.orc_critical_temperature.restype = ctypes.c_double
        L.orc_p_eos.argtypes = [P, ctypes.c_double, ctypes.c_double]
        L.orc_p_eos.restype = ctypes.c_double
        L.orc_psi_squared.argtypes = [P, ctypes.c_double, ctypes.c_double]
        L.orc_psi_squared.restype = ctypes.c_double
        L.orc_equilibrium_moments.argtypes = [ctypes.c_double, dp, dp]
        L.orc_forcing_moments.argtypes = [P, dp, dp, dp, ctypes.c_double, dp]
        L.orc_rho_ave.argtypes = [vp]
        L.orc_rho_ave.restype = ctypes.c_double
        _lib = L
    return _lib


def make_params(**kw) -> OrcParams:
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError(f"unknown oracle parameters: {sorted(unknown)}")
    d.update(kw)
    p = OrcParams()
    for name, _ in _PARAM_FIELDS:
        v = d[name]
        if name == "grav":
            p.grav = (ctypes.c_double * 3)(*[float(x) for x in v])
        else:
            setattr(p, name, v)
    return p


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


class OracleError(RuntimeError):
    pass


class Sim:
    """One oracle simulation.  Fields are numpy arrays of shape (nz, ny, nx)."""

    def __init__(self, **params):
        self.params = dict(DEFAULTS)
        self.params.update(params)
        self._p = make_params(**params)
        self.shape = (self._p.nz, self._p.ny, self._p.nx)
        self.nn = self._p.nx * self._p.ny * self._p.nz
        self.qt = Q19 if self._p.thermal_lattice else Q7  # velocities of the temperature lattice
        h = ctypes.c_void_p()
        rc = lib().orc_create(ctypes.byref(self._p), ctypes.byref(h))
        if rc != 0:
            raise OracleError(f"orc_create failed: {rc}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def init_fields(self, rho, ux, uy, uz, T):
        n = self.nn
        arrs = [_c64(x, n) for x in (rho, ux, uy, uz, T)]
        rc = lib().orc_init_fields(self._h, *[_dp(a) for a in arrs])
        if rc != 0:
            raise OracleError(f"orc_init_fields failed: {rc}")

    def step(self, n=1):
        rc = lib().orc_step(self._h, int(n))
        if rc != 0:
            raise OracleError(f"orc_step failed: {rc}")

    def rho_u_T(self):
        out = [np.empty(self.nn) for _ in range(5)]
        rc = lib().orc_get_rho_u_T(self._h, *[_dp(a) for a in out])
        if rc != 0:
            raise OracleError(f"orc_get_rho_u_T failed: {rc}")
        return tuple(a.reshape(self.shape) for a in out)

    def state(self):
        f = np.empty(Q19 * self.nn)
        g = np.empty(self.qt * self.nn)
        ph = np.empty(self.nn)
        ra = np.empty(1)
        lib().orc_get_state(self._h, _dp(f), _dp(g), _dp(ph), _dp(ra))
        return dict(f=f.reshape((Q19,) + self.shape), g=g.reshape((self.qt,) + self.shape),
                    phi_prev=ph.reshape(self.shape), rho_ave=float(ra[0]))

    def set_state(self, f, g, phi_prev, rho_ave):
        f = _c64(f, Q19 * self.nn)
        g = _c64(g, self.qt * self.nn)
        ph = _c64(phi_prev, self.nn)
        lib().orc_set_state(self._h, _dp(f), _dp(g), _dp(ph), float(rho_ave))

    def reduce(self):
        m = np.empty(1)
        e = np.empty(1)
        lib().orc_reduce(self._h, _dp(m), _dp(e))
        return float(m[0]), float(e[0])

    @property
    def rho_ave(self):
        return lib().orc_rho_ave(self._h)


def tables(**params):
    """Lattice tables as the oracle builds them."""
    p = make_params(**params)
    M = np.empty((Q19, Q19)); Minv = np.empty((Q19, Q19))
    N = np.empty((Q7, Q7)); Ninv = np.empty((Q7, Q7))
    e19 = np.empty((Q19, 3), dtype=np.int32); e7 = np.empty((Q7, 3), dtype=np.int32)
    om = np.empty(Q19); wT = np.empty(Q19)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    lib().orc_tables(ctypes.byref(p), _dp(M), _dp(Minv), _dp(N), _dp(Ninv), ip(e19), ip(e7), _dp(om), _dp(wT))
    wT = wT[:Q19 if p.thermal_lattice else Q7]
    return dict(M=M, Minv=Minv, N=N, Ninv=Ninv, e19=e19, e7=e7, omega=om, wT=wT)


def critical_temperature(**params):
    p = make_params(**params)
    return lib().orc_critical_temperature(ctypes.byref(p))


def p_eos(rho, T, **params):
    p = make_params(**params)
    return lib().orc_p_eos(ctypes.byref(p), float(rho), float(T))


def psi_squared(rho, T, **params):
    p = make_params(**params)
    return lib().orc_psi_squared(ctypes.byref(p), float(rho), float(T))


def equilibrium_moments(rho, u):
    out = np.empty(Q19)
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    lib().orc_equilibrium_moments(float(rho), _dp(uu), _dp(out))
    return out


def forcing_moments(F, Fm, u, psi, **params):
    p = make_params(**params)
    out = np.empty(Q19)
    a = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) for x in (F, Fm, u)]
    lib().orc_forcing_moments(ctypes.byref(p), _dp(a[0]), _dp(a[1]), _dp(a[2]), float(psi), _dp(out))
    return out
