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

def _param_fields(real):
    return [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("bc_z", ctypes.c_int),
        ("a", real), ("b", real), ("R", real), ("acentric", real), ("G", real), ("sigma", real),
        ("tau_e", real), ("tau_v", real), ("tau_q", real), ("tau_pi", real), ("cV", real), ("d", real),
        ("kappa_mode", ctypes.c_int), ("kappa", real), ("vs_q", real), ("vs_pi", real), ("grav", real * 3),
        ("T_wall_patch", real), ("T_wall", real), ("patch_radius", real), ("T_top", real),
        ("thermal", ctypes.c_int), ("bc_T_shell", ctypes.c_int), ("T_shell", real), ("thermal_bgk", ctypes.c_int),
        ("thermal_lattice", ctypes.c_int), ("divu_mode", ctypes.c_int), ("freeze_flow", ctypes.c_int),
        ("wet_mode", ctypes.c_int), ("wet_phi", real), ("wet_phi_in", real), ("wet_drho", real),
        ("wet_square", real), ("wet_disc", real),
    ]


_PARAM_FIELDS = _param_fields(ctypes.c_double)


class OrcParams(ctypes.Structure):
    _fields_ = _PARAM_FIELDS


class OrcParams32(ctypes.Structure):
    """Parameters of the single-precision measurement build (every double a float)."""
    _fields_ = _param_fields(ctypes.c_float)


# Defaults follow Sec. IV: G = -1, acentric factor 0.344, d = 0.95, c_V = 5,
# tau_v = 0.8 (nu = 0.1), tau_e = 1.25, all other relaxation times 1.
DEFAULTS = dict(nx=8, ny=8, nz=8, bc_z=0, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, acentric=0.344,
                G=-1.0, sigma=0.0, tau_e=1.25, tau_v=0.8, tau_q=1.0, tau_pi=1.0, cV=5.0, d=0.95,
                kappa_mode=0, kappa=0.2, vs_q=1.0, vs_pi=1.0, grav=(0.0, 0.0, 0.0),
                T_wall_patch=0.0, T_wall=0.0, patch_radius=0.0, T_top=0.0, thermal=1, bc_T_shell=0, T_shell=0.0,
                thermal_bgk=0, thermal_lattice=0, divu_mode=0, freeze_flow=0,
                wet_mode=0, wet_phi=1.0, wet_phi_in=1.0, wet_drho=0.0, wet_square=0.0, wet_disc=0.0)

_libs = {}


def lib(fp32=False):
    """The FP64 oracle (or, with fp32, the same source built in single
    precision, a measurement of plain FP32 evaluation)."""
    if fp32 in _libs:
        return _libs[fp32]
    path = _build.library(fp32)
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build(fp32=fp32)
    L = ctypes.CDLL(path)
    real = ctypes.c_float if fp32 else ctypes.c_double
    P = ctypes.POINTER(OrcParams32 if fp32 else OrcParams)
    dp = ctypes.POINTER(real)
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
    L.orc_set_state.argtypes = [vp, dp, dp, dp, real]
    L.orc_reduce.argtypes = [vp, dp, dp]
    L.orc_tables.argtypes = [P, dp, dp, dp, dp, ip, ip, dp, dp]
    L.orc_critical_temperature.argtypes = [P]
    L.orc_critical_temperature.restype = real
    L.orc_p_eos.argtypes = [P, real, real]
    L.orc_p_eos.restype = real
    L.orc_psi_squared.argtypes = [P, real, real]
    L.orc_psi_squared.restype = real
    L.orc_equilibrium_moments.argtypes = [real, dp, dp]
    L.orc_forcing_moments.argtypes = [P, dp, dp, dp, real, dp]
    L.orc_rho_ave.argtypes = [vp]
    L.orc_rho_ave.restype = real
    L.orc_max_threads.argtypes = []
    L.orc_max_threads.restype = ctypes.c_int
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = None
    _libs[fp32] = L
    return L


def make_params(fp32=False, **kw):
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError(f"unknown oracle parameters: {sorted(unknown)}")
    d.update(kw)
    p = OrcParams32() if fp32 else OrcParams()
    real = ctypes.c_float if fp32 else ctypes.c_double
    for name, _ in _PARAM_FIELDS:
        v = d[name]
        if name == "grav":
            p.grav = (real * 3)(*[float(x) for x in v])
        else:
            setattr(p, name, v)
    return p


def _dp(a):
    real = ctypes.c_float if a.dtype == np.float32 else ctypes.c_double
    return a.ctypes.data_as(ctypes.POINTER(real))


def _c64(a, n, dtype=np.float64):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype).reshape(-1))
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


class OracleError(RuntimeError):
    pass


class Sim:
    """One oracle simulation.  Fields are numpy arrays of shape (nz, ny, nx).
    fp32=True runs the single-precision measurement build of the same source
    (inputs rounded to FP32, outputs returned as FP64 arrays)."""

    def __init__(self, fp32=False, **params):
        self.params = dict(DEFAULTS)
        self.params.update(params)
        self.fp32 = bool(fp32)
        self._dt = np.float32 if self.fp32 else np.float64
        self._lib = lib(self.fp32)
        self._p = make_params(fp32=self.fp32, **params)
        self.shape = (self._p.nz, self._p.ny, self._p.nx)
        self.nn = self._p.nx * self._p.ny * self._p.nz
        self.qt = Q19 if self._p.thermal_lattice else Q7  # velocities of the temperature lattice
        h = ctypes.c_void_p()
        rc = self._lib.orc_create(ctypes.byref(self._p), ctypes.byref(h))
        if rc != 0:
            raise OracleError(f"orc_create failed: {rc}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _empty(self, n):
        return np.empty(n, dtype=self._dt)

    def init_fields(self, rho, ux, uy, uz, T):
        n = self.nn
        arrs = [_c64(x, n, self._dt) for x in (rho, ux, uy, uz, T)]
        rc = self._lib.orc_init_fields(self._h, *[_dp(a) for a in arrs])
        if rc != 0:
            raise OracleError(f"orc_init_fields failed: {rc}")

    def step(self, n=1):
        rc = self._lib.orc_step(self._h, int(n))
        if rc != 0:
            raise OracleError(f"orc_step failed: {rc}")

    def rho_u_T(self):
        out = [self._empty(self.nn) for _ in range(5)]
        rc = self._lib.orc_get_rho_u_T(self._h, *[_dp(a) for a in out])
        if rc != 0:
            raise OracleError(f"orc_get_rho_u_T failed: {rc}")
        return tuple(a.astype(np.float64, copy=False).reshape(self.shape) for a in out)

    def state(self):
        f = self._empty(Q19 * self.nn)
        g = self._empty(self.qt * self.nn)
        ph = self._empty(self.nn)
        ra = self._empty(1)
        self._lib.orc_get_state(self._h, _dp(f), _dp(g), _dp(ph), _dp(ra))
        return dict(f=f.reshape((Q19,) + self.shape), g=g.reshape((self.qt,) + self.shape),
                    phi_prev=ph.reshape(self.shape), rho_ave=float(ra[0]))

    def set_state(self, f, g, phi_prev, rho_ave):
        f = _c64(f, Q19 * self.nn, self._dt)
        g = _c64(g, self.qt * self.nn, self._dt)
        ph = _c64(phi_prev, self.nn, self._dt)
        self._lib.orc_set_state(self._h, _dp(f), _dp(g), _dp(ph), float(rho_ave))

    def reduce(self):
        m = self._empty(1)
        e = self._empty(1)
        self._lib.orc_reduce(self._h, _dp(m), _dp(e))
        return float(m[0]), float(e[0])

    @property
    def rho_ave(self):
        return self._lib.orc_rho_ave(self._h)


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


def max_threads():
    """OpenMP threads the oracle's parallel passes use in this process."""
    return int(lib().orc_max_threads())


def set_threads(n):
    """OpenMP threads of the oracle's passes in this thread (0: the initial number)."""
    lib().orc_set_threads(int(n))
