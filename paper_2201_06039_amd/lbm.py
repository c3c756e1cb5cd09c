"""Python binding of liblbm (argument marshalling only).

Every step of the path runs in the HIP kernels of liblbm.so; this module
allocates the caller-owned device arena with torch, passes torch's current
HIP stream, and converts numpy arrays to the C-ABI's FP64 host buffers.
There is no fallback: if the library is missing or cannot be loaded, the
import of `Lattice` fails loudly.
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ESTATE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC, BC_WALL_BOTTOM_OPEN_TOP, BC_WALLS = 0, 1, 2
WET_NEUTRAL, WET_VIRTUAL_DENSITY = 0, 1
KAPPA_CONST_LAMBDA, KAPPA_CONST_CHI = 0, 1
STORE_F32, STORE_F64, STORE_F16, STORE_BF16, STORE_F32_DEV = 0, 1, 2, 3, 4
_STORAGE_NAMES = {"f32": STORE_F32, "f64": STORE_F64, "f16": STORE_F16, "bf16": STORE_BF16,
                  "f32dev": STORE_F32_DEV}
STORAGE_FORMATS = tuple(_STORAGE_NAMES)


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("bc_z", ctypes.c_int),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
        ("acentric", ctypes.c_double), ("G", ctypes.c_double), ("sigma", ctypes.c_double),
        ("tau_e", ctypes.c_double), ("tau_v", ctypes.c_double), ("tau_q", ctypes.c_double),
        ("tau_pi", ctypes.c_double), ("cV", ctypes.c_double), ("d", ctypes.c_double),
        ("kappa_mode", ctypes.c_int), ("kappa", ctypes.c_double),
        ("vs_q", ctypes.c_double), ("vs_pi", ctypes.c_double), ("g", ctypes.c_double * 3),
        ("T_wall_patch", ctypes.c_double), ("T_wall", ctypes.c_double),
        ("patch_radius", ctypes.c_double), ("T_top", ctypes.c_double),
        ("thermal", ctypes.c_int), ("storage", ctypes.c_int),
        ("bc_T_shell", ctypes.c_int), ("T_shell", ctypes.c_double), ("thermal_bgk", ctypes.c_int),
        ("thermal_lattice", ctypes.c_int), ("divu_mode", ctypes.c_int),
        ("wet_mode", ctypes.c_int), ("wet_phi", ctypes.c_double), ("wet_phi_in", ctypes.c_double),
        ("wet_drho", ctypes.c_double), ("wet_square", ctypes.c_double), ("wet_disc", ctypes.c_double),
    ]


# Every entry point declared in include/lbm.h.
EXPORTS = ("lbm_arena_bytes", "lbm_create", "lbm_init_fields", "lbm_step", "lbm_get_rho_u_T", "lbm_reduce",
           "lbm_reduce_static",
           "lbm_state_bytes", "lbm_get_state", "lbm_set_state", "lbm_set_launch", "lbm_get_launch",
           "lbm_launches_per_step", "lbm_destroy", "lbm_strerror",
           "lbm_batch_arena_bytes", "lbm_batch_create", "lbm_batch_init_case", "lbm_batch_step",
           "lbm_batch_get_rho_u_T", "lbm_batch_reduce", "lbm_batch_set_launch", "lbm_batch_get_launch",
           "lbm_batch_case_tile", "lbm_fitted_tile", "lbm_batch_autotune", "lbm_batch_destroy", "lbm_copy_probe")

_lib = None


def library_path() -> str:
    """The in-tree build, unless LBM_LIBRARY names another build of liblbm."""
    return os.environ.get("LBM_LIBRARY", _build.LIB)


def load_library():
    """Load liblbm.so (built in-tree by paper_2201_06039_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"liblbm.so not found at {path}; run `python -m paper_2201_06039_amd.build`")
    L = ctypes.CDLL(path)
    vp, dp, P = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(LbmParams)
    ip = ctypes.POINTER(ctypes.c_int)
    L.lbm_arena_bytes.argtypes = [P]
    L.lbm_arena_bytes.restype = ctypes.c_size_t
    L.lbm_create.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbm_init_fields.argtypes = [vp, dp, dp, dp, dp, dp]
    L.lbm_step.argtypes = [vp, ctypes.c_int]
    L.lbm_get_rho_u_T.argtypes = [vp, dp, dp, dp, dp, dp]
    L.lbm_reduce.argtypes = [vp, dp, dp]
    L.lbm_reduce_static.argtypes = [vp, dp, dp]
    L.lbm_state_bytes.argtypes = [vp]
    L.lbm_state_bytes.restype = ctypes.c_size_t
    L.lbm_get_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbm_set_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbm_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.lbm_get_launch.argtypes = [vp, ip, ip, ip, ip]
    L.lbm_launches_per_step.argtypes = [vp]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_strerror.argtypes = [ctypes.c_int]
    L.lbm_strerror.restype = ctypes.c_char_p
    L.lbm_batch_arena_bytes.argtypes = [P, ctypes.c_int]
    L.lbm_batch_arena_bytes.restype = ctypes.c_size_t
    L.lbm_batch_create.argtypes = [P, ctypes.c_int, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbm_batch_init_case.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp, dp]
    L.lbm_batch_step.argtypes = [vp, ctypes.c_int]
    L.lbm_batch_get_rho_u_T.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp, dp]
    L.lbm_batch_reduce.argtypes = [vp, ctypes.c_int, dp, dp]
    L.lbm_batch_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.lbm_batch_get_launch.argtypes = [vp, ip, ip, ip, ip, ip]
    L.lbm_batch_case_tile.argtypes = [vp, ctypes.c_int, ip, ip, ip]
    L.lbm_fitted_tile.argtypes = [ctypes.POINTER(LbmParams), ip, ip]
    L.lbm_batch_autotune.argtypes = [vp, ctypes.c_int, dp]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_destroy.restype = None
    L.lbm_copy_probe.argtypes = [vp, vp, ctypes.c_size_t, vp]
    for name in ("lbm_create", "lbm_init_fields", "lbm_step", "lbm_get_rho_u_T", "lbm_reduce", "lbm_reduce_static",
                 "lbm_get_state",
                 "lbm_set_state", "lbm_set_launch", "lbm_get_launch", "lbm_launches_per_step",
                 "lbm_batch_create", "lbm_batch_init_case", "lbm_batch_step", "lbm_batch_get_rho_u_T",
                 "lbm_batch_reduce", "lbm_batch_set_launch", "lbm_batch_get_launch", "lbm_batch_case_tile",
                 "lbm_fitted_tile",
                 "lbm_batch_autotune", "lbm_copy_probe"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class LbmError(RuntimeError):
    def __init__(self, call, status):
        msg = load_library().lbm_strerror(status).decode()
        super().__init__(f"{call} failed: {status} ({msg})")
        self.status = status


def make_params(params: dict, storage="f32") -> LbmParams:
    p = LbmParams()
    names = [n for n, _ in LbmParams._fields_]
    src = dict(params)
    if "grav" in src and "g" not in src:
        src["g"] = src.pop("grav")
    src.setdefault("storage", _STORAGE_NAMES[storage] if isinstance(storage, str) else storage)
    src.setdefault("bc_T_shell", 0)
    src.setdefault("T_shell", 0.0)
    src.setdefault("thermal_bgk", 0)
    src.setdefault("thermal_lattice", 0)
    src.setdefault("divu_mode", 0)
    src.setdefault("wet_mode", 0)
    src.setdefault("wet_phi", 1.0)
    src.setdefault("wet_phi_in", 1.0)
    src.setdefault("wet_drho", 0.0)
    src.setdefault("wet_square", 0.0)
    src.setdefault("wet_disc", 0.0)
    for n in names:
        if n not in src:
            raise KeyError(f"missing parameter {n!r}")
        v = src[n]
        if n == "g":
            p.g = (ctypes.c_double * 3)(*[float(x) for x in v])
        elif isinstance(getattr(p, n), int):
            setattr(p, n, int(v))
        else:
            setattr(p, n, float(v))
    return p


def arena_bytes(params: dict, storage="f32") -> int:
    return load_library().lbm_arena_bytes(ctypes.byref(make_params(params, storage)))


def fitted_tile(params: dict, storage="f16"):
    """(tile_x, tile_y) of the fitted tile a batch gives this lattice."""
    tx, ty = ctypes.c_int(), ctypes.c_int()
    rc = load_library().lbm_fitted_tile(ctypes.byref(make_params(params, storage)), ctypes.byref(tx), ctypes.byref(ty))
    if rc != OK:
        raise LbmError("lbm_fitted_tile", rc)
    return tx.value, ty.value


def _params_array(cases, storage):
    arr = (LbmParams * len(cases))()
    for i, c in enumerate(cases):
        arr[i] = make_params(c, storage)
    return arr


def batch_arena_bytes(cases, storage="f16") -> int:
    return load_library().lbm_batch_arena_bytes(_params_array(cases, storage), len(cases))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Lattice:
    """One simulation on one GPU.  Host arrays are float64 of shape (nz, ny, nx).

    Work goes to `stream` (torch's current stream by default).  On a stream of
    its own (e.g. torch.cuda.Stream(), default priority) lbm_step replays
    pairs of steps as a captured graph; on the default stream it launches
    them directly."""

    def __init__(self, params: dict, storage="f32", device="cuda", stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self._p = make_params(params, storage)
        self.shape = (self._p.nz, self._p.ny, self._p.nx)
        self.nn = self._p.nx * self._p.ny * self._p.nz
        nbytes = self.lib.lbm_arena_bytes(ctypes.byref(self._p))
        if nbytes == 0:
            raise LbmError("lbm_arena_bytes", EINVAL)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        current = torch.cuda.current_stream(self.arena.device)
        self.stream = stream if stream is not None else current
        if self.stream != current:
            # the arena was allocated on torch's current stream; order the lattice's stream after it
            self.stream.wait_stream(current)
        h = ctypes.c_void_p()
        rc = self.lib.lbm_create(ctypes.byref(self._p), ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != OK:
            raise LbmError("lbm_create", rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            # the arena goes back to torch's allocator: let the lattice's stream finish with it first
            self.stream.synchronize()
            self.lib.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, call, rc):
        if rc != OK:
            raise LbmError(call, rc)

    def init_fields(self, rho, ux, uy, uz, T):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1)) for a in (rho, ux, uy, uz, T)]
        for a in arrs:
            if a.size != self.nn:
                raise ValueError(f"expected {self.nn} values, got {a.size}")
        self._check("lbm_init_fields", self.lib.lbm_init_fields(self._h, *[_dp(a) for a in arrs]))

    def step(self, n=1):
        self._check("lbm_step", self.lib.lbm_step(self._h, int(n)))

    def rho_u_T(self):
        out = [np.empty(self.nn) for _ in range(5)]
        self._check("lbm_get_rho_u_T", self.lib.lbm_get_rho_u_T(self._h, *[_dp(a) for a in out]))
        return tuple(a.reshape(self.shape) for a in out)

    def reduce(self):
        m, e = ctypes.c_double(), ctypes.c_double()
        self._check("lbm_reduce", self.lib.lbm_reduce(self._h, ctypes.byref(m), ctypes.byref(e)))
        return m.value, e.value

    def reduce_static(self):
        """lbm_reduce through the library's static scratch (allocates nothing)."""
        m, e = ctypes.c_double(), ctypes.c_double()
        self._check("lbm_reduce_static", self.lib.lbm_reduce_static(self._h, ctypes.byref(m), ctypes.byref(e)))
        return m.value, e.value

    def state_bytes(self):
        return self.lib.lbm_state_bytes(self._h)

    def get_state(self) -> bytes:
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        self._check("lbm_get_state", self.lib.lbm_get_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
        return buf.tobytes()

    def set_state(self, blob: bytes):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        self._check("lbm_set_state", self.lib.lbm_set_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))

    def set_launch(self, tile_x, tile_y, chunk_z):
        self._check("lbm_set_launch", self.lib.lbm_set_launch(self._h, tile_x, tile_y, chunk_z))

    def launch(self):
        v = [ctypes.c_int() for _ in range(4)]
        self._check("lbm_get_launch", self.lib.lbm_get_launch(self._h, *[ctypes.byref(x) for x in v]))
        return dict(tile_x=v[0].value, tile_y=v[1].value, chunk_z=v[2].value, workgroups=v[3].value)

    def launches_per_step(self):
        return self.lib.lbm_launches_per_step(self._h)


class Batch:
    """Many independent lattices advanced by one launch per time step.

    `cases` is a list of parameter dicts (periodic, no gravity, one storage
    format for all).  The batch runs on a stream of its own (default
    priority) so that lbm_batch_step can replay captured graphs; readouts
    synchronise it."""

    def __init__(self, cases, storage="f16", device="cuda", stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self._params = _params_array(cases, storage)
        self.n = len(cases)
        self.shapes = [(p.nz, p.ny, p.nx) for p in self._params]
        nbytes = self.lib.lbm_batch_arena_bytes(self._params, self.n)
        if nbytes == 0:
            raise LbmError("lbm_batch_arena_bytes", EINVAL)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.arena.device)
        # the arena was allocated on torch's current stream; order the batch's stream after it
        self.stream.wait_stream(torch.cuda.current_stream(self.arena.device))
        h = ctypes.c_void_p()
        rc = self.lib.lbm_batch_create(self._params, self.n, ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != OK:
            raise LbmError("lbm_batch_create", rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            # the arena goes back to torch's allocator: let the batch's stream finish with it first
            self.stream.synchronize()
            self.lib.lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, call, rc):
        if rc != OK:
            raise LbmError(call, rc)

    def init_case(self, c, rho, ux, uy, uz, T):
        nn = int(np.prod(self.shapes[c]))
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1)) for a in (rho, ux, uy, uz, T)]
        for a in arrs:
            if a.size != nn:
                raise ValueError(f"case {c}: expected {nn} values, got {a.size}")
        self._check("lbm_batch_init_case", self.lib.lbm_batch_init_case(self._h, int(c), *[_dp(a) for a in arrs]))

    def step(self, n=1):
        self._check("lbm_batch_step", self.lib.lbm_batch_step(self._h, int(n)))

    def rho_u_T(self, c):
        nn = int(np.prod(self.shapes[c]))
        out = [np.empty(nn) for _ in range(5)]
        self._check("lbm_batch_get_rho_u_T", self.lib.lbm_batch_get_rho_u_T(self._h, int(c), *[_dp(a) for a in out]))
        return tuple(a.reshape(self.shapes[c]) for a in out)

    def reduce(self, c):
        m, e = ctypes.c_double(), ctypes.c_double()
        self._check("lbm_batch_reduce", self.lib.lbm_batch_reduce(self._h, int(c), ctypes.byref(m), ctypes.byref(e)))
        return m.value, e.value

    def set_launch(self, tile_x, tile_y, chunk_z, workgroups=0):
        self._check("lbm_batch_set_launch", self.lib.lbm_batch_set_launch(self._h, tile_x, tile_y, chunk_z,
                                                                          workgroups))

    def launch(self):
        v = [ctypes.c_int() for _ in range(5)]
        self._check("lbm_batch_get_launch", self.lib.lbm_batch_get_launch(self._h, *[ctypes.byref(x) for x in v]))
        return dict(tile_x=v[0].value, tile_y=v[1].value, chunk_z=v[2].value, workgroups=v[3].value,
                    items=v[4].value)

    def case_tile(self, c):
        """(tile_x, tile_y, threads per workgroup) of lattice c under the current launch."""
        v = [ctypes.c_int() for _ in range(3)]
        self._check("lbm_batch_case_tile", self.lib.lbm_batch_case_tile(self._h, int(c), *[ctypes.byref(x) for x in v]))
        return v[0].value, v[1].value, v[2].value

    def autotune(self, steps=10):
        ms = ctypes.c_double()
        self._check("lbm_batch_autotune", self.lib.lbm_batch_autotune(self._h, int(steps), ctypes.byref(ms)))
        return ms.value


def copy_probe(src, dst, stream=None):
    """Enqueue the library's streaming copy of torch tensor `src` into `dst`
    (same byte size, a multiple of 16) on `stream` (torch's current stream by
    default)."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy_probe: tensors of different byte size")
    stream = stream if stream is not None else torch.cuda.current_stream(src.device)
    rc = load_library().lbm_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                                       ctypes.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise LbmError("lbm_copy_probe", rc)
