"""Sessile-droplet geometry for the wettability pins (test infrastructure).

A half-cylinder of liquid on the bottom wall of a quasi-2D box, and the
contact angle of a 2D density field: a least-squares circle through the
half-density contour (away from the wall rows), with the wall plane at
z = -1/2 (halfway bounce-back).  The angle is measured inside the liquid:
90 degrees for a circle centred on the wall plane.
"""
import numpy as np


def half_cylinder(nx, nz, r0, rho_l, rho_g, T, width=4.0):
    """rho, ux, uy, uz, T of shape (nz, 1, nx): a tanh half-cylinder of radius
    r0 centred at x = (nx - 1)/2 on the wall plane z = -1/2."""
    x = np.arange(nx)[None, :]
    z = np.arange(nz)[:, None]
    r = np.sqrt((x - 0.5 * (nx - 1)) ** 2 + (z + 0.5) ** 2)
    rho = (0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2.0 * (r - r0) / width))[:, None, :]
    zero = np.zeros_like(rho)
    return rho, zero, zero.copy(), zero.copy(), np.full_like(rho, T)


def contact_angle_2d(rho, level, skip_rows=3):
    """Contact angle (degrees) of the level-`level` contour of rho[z, x]."""
    nz, nx = rho.shape
    pts = []
    for z in range(skip_rows, nz):
        row = rho[z] - level
        for x in range(nx - 1):
            if row[x] * row[x + 1] < 0:
                pts.append((x + row[x] / (row[x] - row[x + 1]), z))
    for x in range(nx):
        col = rho[:, x] - level
        for z in range(skip_rows, nz - 1):
            if col[z] * col[z + 1] < 0:
                pts.append((x, z + col[z] / (col[z] - col[z + 1])))
    P = np.array(pts, dtype=float)
    if len(P) < 5:
        raise ValueError("no contour to fit")
    M = np.c_[P[:, 0], P[:, 1], np.ones(len(P))]
    D, E, F = np.linalg.lstsq(M, -(P[:, 0] ** 2 + P[:, 1] ** 2), rcond=None)[0]
    xc, zc = -D / 2.0, -E / 2.0
    Rc = np.sqrt(xc * xc + zc * zc - F)
    return float(np.degrees(np.arccos(np.clip(-(zc + 0.5) / Rc, -1.0, 1.0))))
