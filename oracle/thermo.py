"""Peng-Robinson thermodynamics for the oracle (test infrastructure only).

* `pressure`      -- Eq. (49) of the paper, in numpy.
* `maxwell`       -- liquid/vapour coexistence densities at temperature T by
                     the equal-area rule  int_{rho_g}^{rho_l} (p - p_s)/rho^2
                     drho = 0 with p(rho_g) = p(rho_l) = p_s, evaluated with
                     adaptive quadrature.
* `ln_fugacity`   -- the textbook closed-form PR fugacity coefficient.  Equal
                     fugacities of the two phases is an independent statement
                     of phase equilibrium, used to pin `maxwell`.
"""
import math

import numpy as np
from scipy import integrate, optimize

SQRT2 = math.sqrt(2.0)


def critical_temperature(a, b, R):
    """Sec. IV A: a = 0.45724 R^2 Tc^2/pc, b = 0.0778 R Tc/pc."""
    return 0.0778 / 0.45724 * a / (b * R)


def vartheta(T, Tc, acentric):
    """Eq. (49): temperature function of the attraction term."""
    kappa = 0.37464 + 1.54226 * acentric - 0.26992 * acentric ** 2
    return (1.0 + kappa * (1.0 - math.sqrt(T / Tc))) ** 2


def pressure(rho, T, a, b, R, acentric):
    """Eq. (49) Peng-Robinson EOS (vectorised over rho)."""
    rho = np.asarray(rho, dtype=np.float64)
    Tc = critical_temperature(a, b, R)
    th = vartheta(T, Tc, acentric)
    return rho * R * T / (1.0 - b * rho) - a * th * rho ** 2 / (1.0 + 2.0 * b * rho - b * b * rho ** 2)


def _spinodals(T, a, b, R, acentric):
    """Densities of the local maximum (vapour side) and local minimum (liquid
    side) of p(rho) below the critical temperature."""
    rho = np.linspace(1e-6, 0.999 / b, 40001)
    p = pressure(rho, T, a, b, R, acentric)
    dp = np.diff(p)
    sign = np.sign(dp)
    idx = np.nonzero(sign[:-1] != sign[1:])[0]
    if len(idx) < 2:
        raise ValueError("no two-phase region at this temperature")

    def dpdrho(r):
        h = 1e-7 * max(1.0, r)
        return (pressure(r + h, T, a, b, R, acentric) - pressure(r - h, T, a, b, R, acentric)) / (2 * h)

    r1 = optimize.brentq(dpdrho, rho[idx[0]], rho[idx[0] + 2], xtol=1e-14)
    r2 = optimize.brentq(dpdrho, rho[idx[1]], rho[idx[1] + 2], xtol=1e-14)
    return r1, r2


def maxwell(T, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, acentric=0.344):
    """Coexistence (rho_g, rho_l, p_sat) at temperature T by Maxwell's rule."""
    rs1, rs2 = _spinodals(T, a, b, R, acentric)
    p_hi = float(pressure(rs1, T, a, b, R, acentric))
    p_lo = max(float(pressure(rs2, T, a, b, R, acentric)), 1e-14)

    def branch_roots(ps):
        f = lambda r: float(pressure(r, T, a, b, R, acentric)) - ps
        rg = optimize.brentq(f, 1e-12, rs1, xtol=1e-15, rtol=1e-15)
        rl = optimize.brentq(f, rs2, 0.999999 / b, xtol=1e-15, rtol=1e-15)
        return rg, rl

    def area(ps):
        rg, rl = branch_roots(ps)
        val, _ = integrate.quad(lambda r: (float(pressure(r, T, a, b, R, acentric)) - ps) / r ** 2, rg, rl,
                                epsabs=1e-14, epsrel=1e-13, limit=400)
        return val

    span = p_hi - p_lo
    ps = optimize.brentq(area, p_lo + 1e-9 * span, p_hi - 1e-9 * span, xtol=1e-16, rtol=1e-15)
    rg, rl = branch_roots(ps)
    return rg, rl, ps


def ln_fugacity(rho, T, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, acentric=0.344):
    """Textbook Peng-Robinson fugacity coefficient ln(phi) of a phase of
    density rho at temperature T:
        ln phi = Z - 1 - ln(Z - B) - A/(2 sqrt2 B) ln[(Z + (1+sqrt2)B)/(Z + (1-sqrt2)B)]
    with Z = p/(rho R T), A = a vartheta p/(R T)^2, B = b p/(R T)."""
    Tc = critical_temperature(a, b, R)
    p = float(pressure(rho, T, a, b, R, acentric))
    Z = p / (rho * R * T)
    A = a * vartheta(T, Tc, acentric) * p / (R * T) ** 2
    B = b * p / (R * T)
    return Z - 1.0 - math.log(Z - B) - A / (2.0 * SQRT2 * B) * math.log(
        (Z + (1.0 + SQRT2) * B) / (Z + (1.0 - SQRT2) * B))
