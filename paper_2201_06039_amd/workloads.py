"""Seeded synthetic initial fields for the benchmark workloads and tests.

This module holds geometry and noise only: tanh interface profiles, droplet
placements and a counter-based SplitMix64 noise source.  It contains none of
the lattice Boltzmann arithmetic; the coexistence densities, temperatures and
model parameters of each workload are plain numbers stored in
``workloads.json`` beside this file.

Every generator returns float64 numpy arrays of shape (nz, ny, nx) with node
index i = x + nx*(y + ny*z), i.e. x fastest.
"""
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
WORKLOADS_JSON = os.path.join(_HERE, "workloads.json")

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs k = offset .. offset+count-1 of SplitMix64 (Steele, Lea & Flood,
    2014) started from state `seed`: x_k = seed + (k+1)*golden, then the
    published 64-bit finaliser."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_noise(seed: int, count: int, amplitude: float) -> np.ndarray:
    """Uniform noise in [-amplitude, amplitude) from the top 53 bits of
    SplitMix64, one draw per node index."""
    u = (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (2.0 * u - 1.0) * amplitude


def tanh_blend(dist: np.ndarray, inside: float, outside: float, width: float) -> np.ndarray:
    """inside for dist << 0, outside for dist >> 0; tanh profile of the given width."""
    return 0.5 * (inside + outside) - 0.5 * (inside - outside) * np.tanh(2.0 * dist / width)


def _coords(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def droplet(nx, ny, nz, radius, rho_l, rho_g, T_l, T_v, width=2.0, center=None, noise=0.0, seed=0):
    """Spherical droplet (or, with nz == 1, a cylinder along z) on a periodic
    grid: density and temperature both follow the tanh profile of the radial
    distance.  Optional SplitMix64 density noise."""
    if center is None:
        center = (nx / 2.0, ny / 2.0, nz / 2.0)
    x, y, z = _coords(nx, ny, nz)
    if nz == 1:
        r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2)
    else:
        r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    rho = tanh_blend(r - radius, rho_l, rho_g, width)
    T = tanh_blend(r - radius, T_l, T_v, width)
    if noise:
        rho = rho + uniform_noise(seed, rho.size, noise).reshape(rho.shape)
    zero = np.zeros_like(rho)
    return rho, zero, zero.copy(), zero.copy(), T


def flat_interface(nx, ny, nz, rho_l, rho_g, T, width=2.0, liquid_fraction=0.5):
    """Liquid slab centred in z between two flat interfaces (periodic z)."""
    x, y, z = _coords(nx, ny, nz)
    half = 0.5 * liquid_fraction * nz
    dist = np.abs(z - 0.5 * (nz - 1)) - half
    rho = tanh_blend(dist, rho_l, rho_g, width)
    zero = np.zeros_like(rho)
    return rho, zero, zero.copy(), zero.copy(), np.full_like(rho, T)


def pool(nx, ny, nz, depth, rho_l, rho_g, T, width=2.0, noise=0.0, seed=0):
    """Liquid pool filling z < depth under its vapour, uniform temperature."""
    x, y, z = _coords(nx, ny, nz)
    rho = tanh_blend(z - depth, rho_l, rho_g, width)
    if noise:
        rho = rho + uniform_noise(seed, rho.size, noise).reshape(rho.shape)
    zero = np.zeros_like(rho)
    return rho, zero, zero.copy(), zero.copy(), np.full_like(rho, T)


def multi_droplet(n, count, rmin, rmax, rho_l, rho_g, T, width=2.0, gap=4.0, seed=0):
    """`count` droplets with radii U[rmin, rmax] at SplitMix64-drawn centres in
    a periodic n^3 box, kept `gap` apart (minimum image); the density is the
    maximum of the individual tanh profiles."""
    draws = splitmix64(seed, 4 * count * 64)
    u = (draws >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    centres, radii = [], []
    k = 0
    while len(centres) < count and k + 4 <= u.size:
        c = u[k:k + 3] * n
        r = rmin + (rmax - rmin) * u[k + 3]
        k += 4
        ok = True
        for c2, r2 in zip(centres, radii):
            d = np.abs(c - c2)
            d = np.minimum(d, n - d)
            if np.sqrt((d ** 2).sum()) < r + r2 + gap:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(r)
    rho = np.full((n, n, n), rho_g)
    # A droplet's profile equals rho_g to the last bit once tanh(2 d / width)
    # rounds to 1 (d >= 10 width), so each droplet is evaluated only inside
    # the periodic box of half-side r + 10 width + 1 around its centre.
    reach = 10.0 * width + 1.0
    for c, r in zip(centres, radii):
        ax = []
        for k in range(3):
            lo = int(np.floor(c[k] - r - reach))
            idx = np.arange(lo, int(np.ceil(c[k] + r + reach)) + 1)
            if idx.size >= n:
                idx = np.arange(n)
            d = np.abs(np.mod(idx, n) - c[k])
            ax.append((np.mod(idx, n), np.minimum(d, n - d)))
        (ix, dx), (iy, dy), (iz, dz) = ax
        dist = np.sqrt(dx[None, None, :] ** 2 + dy[None, :, None] ** 2 + dz[:, None, None] ** 2) - r
        box = np.ix_(iz, iy, ix)
        rho[box] = np.maximum(rho[box], tanh_blend(dist, rho_l, rho_g, width))
    zero = np.zeros_like(rho)
    return rho, zero, zero.copy(), zero.copy(), np.full_like(rho, T)


def load(name: str) -> dict:
    """Parameters and initial-condition numbers of a named workload."""
    with open(WORKLOADS_JSON) as fh:
        table = json.load(fh)
    if name not in table["workloads"]:
        raise KeyError(f"unknown workload {name!r}; have {sorted(table['workloads'])}")
    return table["workloads"][name]


def fields(w: dict):
    """Initial (rho, ux, uy, uz, T) for a workload record from `load`."""
    kind = w["init"]["kind"]
    a = dict(w["init"])
    a.pop("kind")
    nx, ny, nz = w["params"]["nx"], w["params"]["ny"], w["params"]["nz"]
    if kind == "droplet":
        return droplet(nx, ny, nz, **a)
    if kind == "flat":
        return flat_interface(nx, ny, nz, **a)
    if kind == "pool":
        return pool(nx, ny, nz, **a)
    if kind == "multi_droplet":
        assert nx == ny == nz
        return multi_droplet(nx, **a)
    raise ValueError(kind)
