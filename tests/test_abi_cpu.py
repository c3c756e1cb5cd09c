"""The C-ABI library loads on the CPU, exports every symbol include/lbm.h
declares, and validates parameters without touching a GPU."""
import ctypes
import os
import re

import pytest

from conftest import ROOT


@pytest.fixture(scope="module")
def lib():
    from paper_2201_06039_amd import build, lbm
    if not build.up_to_date():
        build.build()
    return lbm.load_library()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("lbm_create", "lbm_init_fields", "lbm_step", "lbm_get_rho_u_T", "lbm_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2201_06039_amd import lbm
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(lbm.EXPORTS) == declared_functions()


def test_params_struct_matches_the_header(tmp_path):
    """The binding's lbm_params has the C struct's size and every field at
    its C offset (include/lbm.h compiled with the host C compiler)."""
    import shutil
    import subprocess
    from paper_2201_06039_amd import lbm
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = [f[0] for f in lbm.LbmParams._fields_]
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\nint main(void) {\n'
           '    printf("%zu\\n", sizeof(lbm_params));\n' +
           "".join(f'    printf("%zu\\n", offsetof(lbm_params, {f}));\n' for f in fields) + "    return 0;\n}\n")
    (tmp_path / "offsets.c").write_text(src)
    exe = str(tmp_path / "offsets")
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), "-o", exe, str(tmp_path / "offsets.c")], check=True)
    out = [int(v) for v in subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(lbm.LbmParams)
    for f, off in zip(fields, out[1:]):
        assert getattr(lbm.LbmParams, f).offset == off, f


def _fitted_rule(nx, ny):
    """The selection the batch documents, written out: of the tiles with
    256..512 nodes whose extended tile fits 700 LDS nodes and that are exactly
    nx wide (nx <= 128) or 4k wide from 64 to below nx (and 128 at most), the
    one with the fewest idle slots of 512-thread workgroups; within 2% of it
    the smaller halo (two rows for whole-row tiles), then the wider tile."""
    import math
    widths = ([nx] if 2 <= nx <= 128 else []) + [t for t in range(64, 129, 4) if t < nx]
    best, be, bh = (32, 16), -1.0, 1 << 30
    for tx in widths:
        for ty in range(1, 257):
            if not 256 <= tx * ty <= 512 or (tx + 2) * (ty + 2) > 700:
                continue
            e = nx * ny / (math.ceil(nx / tx) * math.ceil(ny / ty) * 512)
            halo = 2 * tx if tx == nx else 2 * (tx + ty) + 4
            if e > be + 0.02 or (e > be - 0.02 and (halo < bh or (halo == bh and tx > best[0]))):
                best, be, bh = (tx, ty), max(be, e), halo
    return best


def test_fitted_tiles_on_the_host(lib):
    """The fitted tile of every lattice of the 256-lattice batch, computed on
    the host (no device): it follows the documented rule, and the batch's
    thread slots hold nodes with the efficiency the batch reports (0.890)."""
    import math
    from paper_2201_06039_amd import lbm, workloads as W
    cases = W.load("batch_256")["cases"]
    nodes = slots = 0
    for c in cases:
        p = c["params"]
        nx, ny, nz = p["nx"], p["ny"], p["nz"]
        tx, ty = lbm.fitted_tile(p, "f16")
        assert 256 <= tx * ty <= 512 and (tx + 2) * (ty + 2) <= 700, (nx, tx, ty)
        assert tx == nx or (tx % 4 == 0 and 64 <= tx < nx), (nx, tx)
        assert (tx, ty) == _fitted_rule(nx, ny), (nx, ny, tx, ty)
        nodes += nx * ny * nz
        slots += math.ceil(nx / tx) * math.ceil(ny / ty) * 512 * nz
    assert abs(nodes / slots - 0.8904) < 5e-4
    # other sizes: odd, narrow, wider than 128, ragged
    for nx, ny in ((17, 33), (85, 20), (150, 9), (200, 200), (2, 300)):
        p = dict(cases[0]["params"], nx=nx, ny=ny, nz=8)
        assert lbm.fitted_tile(p, "f16") == _fitted_rule(nx, ny), (nx, ny)
    with pytest.raises(lbm.LbmError):
        lbm.fitted_tile(cases[0]["params"], "f64")


def test_arena_bytes_and_validation(lib):
    from paper_2201_06039_amd import lbm, workloads as W
    p = W.load("evaporation_128")["params"]
    n = 128 ** 3
    b32 = lbm.arena_bytes(p, "f32")
    b64 = lbm.arena_bytes(p, "f64")
    # two copies of 26 populations + history + 6 FP64 staging planes
    assert b32 >= (2 * 26 + 1) * 4 * n + 6 * 8 * n
    assert b64 >= (2 * 26 + 1) * 8 * n + 6 * 8 * n
    assert b32 < 1.01 * ((2 * 26 + 1) * 4 * n + 6 * 8 * n) + (1 << 22)
    for bad in (dict(tau_e=0.5), dict(nx=0), dict(kappa=0.0), dict(d=1.0), dict(G=0.0), dict(bc_z=1, nz=2),
                dict(vs_q=0.4), dict(thermal=2), dict(storage=7)):
        q = dict(p)
        q.update(bad)
        assert lbm.arena_bytes(q) == 0, bad


def test_arena_bytes_of_the_storage_formats(lib):
    """Deviation formats hold 26 population planes of 2 bytes (f16, bf16) or
    4 bytes (f32dev) and two reference planes (rho_r, T_r: FP16 for f16,
    FP32 otherwise) per copy."""
    from paper_2201_06039_amd import lbm, workloads as W
    p = W.load("evaporation_128")["params"]
    n = 128 ** 3
    rest = 4 * n + 6 * 8 * n  # FP32 phi history + FP64 staging
    for fmt, es, refs in (("f16", 2, 2 * 2), ("bf16", 2, 2 * 4), ("f32dev", 4, 2 * 4), ("f32", 4, 0)):
        copy = (26 * es + refs) * n
        b = lbm.arena_bytes(p, fmt)
        assert 2 * copy + rest <= b < 2 * copy + rest + (1 << 22), fmt
    assert set(lbm.STORAGE_FORMATS) == {"f32", "f64", "f16", "bf16", "f32dev"}


def test_reservoir_boundary_validation(lib):
    """The constant-temperature layer needs a periodic grid, a live
    temperature lattice and a positive temperature."""
    from paper_2201_06039_amd import lbm, workloads as W
    p = dict(W.load("d2_law_48")["params"])
    assert lbm.arena_bytes(p) > 0
    for bad in (dict(bc_z=1), dict(thermal=0), dict(T_shell=0.0), dict(bc_T_shell=2)):
        q = dict(p)
        q.update(bad)
        assert lbm.arena_bytes(q) == 0, bad


def test_create_rejects_bad_arguments_before_any_device_call(lib):
    from paper_2201_06039_amd import lbm, workloads as W
    p = dict(W.load("static_droplet_32")["params"])
    h = ctypes.c_void_p()
    cp = lbm.make_params(p)
    # NULL arena
    assert lib.lbm_create(ctypes.byref(cp), None, 1 << 30, None, ctypes.byref(h)) == lbm.EINVAL
    # arena too small (the pointer is never dereferenced on this path)
    assert lib.lbm_create(ctypes.byref(cp), ctypes.c_void_p(256), 1024, None, ctypes.byref(h)) == lbm.ENOMEM
    # misaligned arena
    need = lib.lbm_arena_bytes(ctypes.byref(cp))
    assert lib.lbm_create(ctypes.byref(cp), ctypes.c_void_p(257), need, None, ctypes.byref(h)) == lbm.ENOMEM
    p["tau_v"] = 0.3
    assert lib.lbm_create(ctypes.byref(lbm.make_params(p)), ctypes.c_void_p(256), 1 << 40, None,
                          ctypes.byref(h)) == lbm.EINVAL
    assert lib.lbm_step(None, 1) == lbm.EINVAL
    lib.lbm_destroy(None)


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, 17):
        assert isinstance(lib.lbm_strerror(code), bytes)


def test_batch_validation(lib):
    """A batch takes periodic lattices without gravity, all in one storage
    format; its arena holds every lattice's own regions."""
    from paper_2201_06039_amd import lbm, workloads as W
    a = dict(W.load("static_droplet_32")["params"])
    b = dict(a, nx=24, ny=20, nz=18)
    c = dict(W.load("d2_law_48")["params"])
    good = lbm.batch_arena_bytes([a, b, c], "f16")
    assert good > lbm.arena_bytes(a, "f16") + lbm.arena_bytes(b, "f16") - 2 * 6 * 8 * 32 ** 3
    assert lbm.batch_arena_bytes([a], "f32") > 0
    assert lbm.batch_arena_bytes([], "f16") == 0
    walls = dict(W.load("pool_boiling_32x32x48")["params"], grav=[0.0, 0.0, 0.0])
    gravity = dict(a, grav=[0.0, 0.0, -1e-5])
    for bad in ([a, walls], [a, gravity], [a, dict(a, tau_v=0.4)]):
        assert lbm.batch_arena_bytes(bad, "f16") == 0
    p = lbm._params_array([a, b], "f16")
    p[1].storage = lbm.STORE_F32
    assert lib.lbm_batch_arena_bytes(p, 2) == 0
    h = ctypes.c_void_p()
    assert lib.lbm_batch_create(p, 2, ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(h)) == lbm.EINVAL
    assert lib.lbm_batch_step(None, 1) == lbm.EINVAL
    lib.lbm_batch_destroy(None)



def test_d3q19_temperature_lattice_arena_and_validation(lib):
    """The D3Q19 temperature lattice stores 19 g planes (38 population planes
    per copy); it takes the BGK collision, the F32, F64 and F16 formats, and
    no batches."""
    from paper_2201_06039_amd import lbm, workloads as W
    p = dict(W.load("evaporation_128")["params"], thermal_lattice=1, thermal_bgk=1)
    n = 128 ** 3
    for fmt, es, refs, cs in (("f16", 2, 2 * 2, 4), ("f32", 4, 0, 4), ("f64", 8, 0, 8)):
        copy = (38 * es + refs) * n
        rest = cs * n + 6 * 8 * n
        b = lbm.arena_bytes(p, fmt)
        assert 2 * copy + rest <= b < 2 * copy + rest + (1 << 22), fmt
        assert b > lbm.arena_bytes(dict(p, thermal_lattice=0), fmt)
    for fmt in ("bf16", "f32dev"):
        assert lbm.arena_bytes(p, fmt) == 0, fmt
    for bad in (dict(thermal_bgk=0), dict(thermal_lattice=2), dict(thermal_lattice=-1)):
        assert lbm.arena_bytes(dict(p, **bad)) == 0, bad
    a = dict(W.load("static_droplet_32")["params"])
    assert lbm.batch_arena_bytes([a, a], "f16") > 0
    assert lbm.batch_arena_bytes([a, dict(a, thermal_lattice=1, thermal_bgk=1)], "f16") == 0


def test_divergence_mode_validation(lib):
    """div u of Eq. (48) (LBM_DIVU_LOCAL) or by finite differences
    (LBM_DIVU_FD); the finite-difference form is not built into batches."""
    from paper_2201_06039_amd import lbm, workloads as W
    p = dict(W.load("static_droplet_32")["params"])
    assert lbm.arena_bytes(dict(p, divu_mode=1)) == lbm.arena_bytes(p) > 0
    assert lbm.arena_bytes(dict(p, divu_mode=2)) == 0
    assert lbm.arena_bytes(dict(p, divu_mode=-1)) == 0
    assert lbm.batch_arena_bytes([p, dict(p, divu_mode=1)], "f16") == 0
    for fmt in ("f32", "f64", "f16"):
        assert lbm.arena_bytes(dict(p, divu_mode=1), fmt) > 0, fmt
    for fmt in ("bf16", "f32dev"):
        assert lbm.arena_bytes(dict(p, divu_mode=1), fmt) == 0, fmt


def test_large_grid_limits(lib):
    """Grids beyond the 4 GiB reach of a buffer resource are valid (their
    copies are addressed with 64-bit plain pointers): a 1024 x 1024 x 600
    FP32 grid needs two copies of 13 pair planes of 8 bytes a node plus the
    reference-free tail, far past 2^32 bytes.  The limits that remain: the
    grid's elements of one plane kind must span under 2^32 bytes, and so must
    an x-y plane of the paired layout."""
    from paper_2201_06039_amd import lbm, workloads as W
    p = dict(W.load("static_droplet_32")["params"])
    n = 1024 * 1024 * 600
    big = dict(p, nx=1024, ny=1024, nz=600)
    b = lbm.arena_bytes(big, "f32")
    stride = -(-n // 128) * 128
    assert b >= 2 * 26 * 4 * stride + 4 * n + 6 * 8 * n
    assert b < 2 * 26 * 4 * stride + 4 * n + 6 * 8 * n + (1 << 27)  # + per-workgroup partial sums
    assert lbm.arena_bytes(dict(p, nx=1024, ny=1024, nz=1100), "f16") > 0   # 2^30 < n < 2^31 for 2-byte elements
    assert lbm.arena_bytes(dict(p, nx=1024, ny=1024, nz=1024), "f32") == 0  # n * 4 bytes reaches 2^32
    assert lbm.arena_bytes(dict(p, nx=1024, ny=1024, nz=2048), "f16") == 0  # n * 2 bytes reaches 2^32
    assert lbm.arena_bytes(dict(p, nx=1 << 15, ny=1 << 14, nz=1), "f16") == 0  # one paired plane reaches 2^32
