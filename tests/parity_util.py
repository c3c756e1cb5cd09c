"""Helpers shared by the GPU parity tests: run the HIP path (through the
C-ABI) and the FP64 oracle on the same seeded inputs and compare them."""
import copy

import numpy as np

from paper_2201_06039_amd import workloads as W


def workload(name, **overrides):
    w = copy.deepcopy(W.load(name))
    init_keys = set(w["init"])
    for k, v in overrides.items():
        if k in init_keys:
            w["init"][k] = v
        else:
            w["params"][k] = v
    return w


def run_gpu(w, steps, storage="f32", launch=None, fields=None, chunks=None):
    """Run `steps` steps on cuda:0; `chunks` splits them into several calls."""
    from paper_2201_06039_amd import lbm
    lat = lbm.Lattice(w["params"], storage=storage, device="cuda:0")
    if launch:
        lat.set_launch(*launch)
    lat.init_fields(*(fields if fields is not None else W.fields(w)))
    for n in (chunks or [steps]):
        lat.step(n)
    out = lat.rho_u_T()
    lat.close()
    return out


def run_oracle(w, steps, fields=None):
    from oracle import sim
    s = sim.Sim(**w["params"])
    s.init_fields(*(fields if fields is not None else W.fields(w)))
    s.step(steps)
    out = s.rho_u_T()
    s.close()
    return out


def errors(got, ref):
    """rel(X) = max|X - X_ref| / max|X_ref| for rho and T;
    u: max |u - u_ref|_2 / max |u_ref|_2."""
    rho, ux, uy, uz, T = got
    r_rho, r_ux, r_uy, r_uz, r_T = ref
    e = {}
    e["rho"] = float(np.abs(rho - r_rho).max() / np.abs(r_rho).max())
    e["T"] = float(np.abs(T - r_T).max() / np.abs(r_T).max())
    du = np.sqrt((ux - r_ux) ** 2 + (uy - r_uy) ** 2 + (uz - r_uz) ** 2)
    un = np.sqrt(r_ux ** 2 + r_uy ** 2 + r_uz ** 2)
    e["u"] = float(du.max() / un.max())
    e["u_l2"] = float(np.sqrt((du ** 2).sum() / (un ** 2).sum()))
    return e


def block_oracle(w, fields, nodes, steps, half=8):
    """The oracle's rho, u, T after `steps` steps at individual nodes of a
    periodic grid, each from its own (2 half)^3 block of the initial fields
    cut around the node (periodic indices).  A step reaches two nodes out
    (the streaming and the 18-neighbour stencils) and the readout velocity one
    more, so the block centre is exact while 2 steps + 2 <= half (no gravity:
    rho_ave does not enter).  `nodes` is a list of (z, y, x); returns five
    arrays of len(nodes)."""
    from oracle import sim
    assert 2 * steps + 2 <= half, "block too small for the step count"
    nz, ny, nx = fields[0].shape
    p = dict(w["params"], nx=2 * half, ny=2 * half, nz=2 * half)
    assert p.get("bc_z", 0) == 0 and not p.get("bc_T_shell", 0) and not any(p.get("grav", (0, 0, 0)))
    out = np.empty((5, len(nodes)))
    for k, (z, y, x) in enumerate(nodes):
        iz = np.arange(z - half, z + half) % nz
        iy = np.arange(y - half, y + half) % ny
        ix = np.arange(x - half, x + half) % nx
        blk = [f[np.ix_(iz, iy, ix)] for f in fields]
        s = sim.Sim(**p)
        s.init_fields(*blk)
        s.step(steps)
        r = s.rho_u_T()
        s.close()
        for c in range(5):
            out[c, k] = r[c][half, half, half]
    return out


def sample_errors(got, ref):
    """errors() restricted to sampled nodes: got and ref are (5, n) arrays."""
    return errors(tuple(got), tuple(ref))
