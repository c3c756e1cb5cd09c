"""Derived quantities used to compare the storage formats with the FP64
oracle: the coexistence densities of a flat slab, the Laplace pressure jump of
a static droplet, and the D^2 slope of an evaporating droplet (Sec. IV A).

Each case is a workload, a set of overrides and a step schedule; `measure`
reduces a run's (rho, u, T) output to the case's numbers.  The same reduction
is applied to the oracle's output (tests/golden/make_precision_refs.py) and to
the GPU output (tests/test_gpu_precision.py)."""
import copy

import numpy as np

from paper_2201_06039_amd import workloads as W

CASES = {
    # isothermal flat slab, 2 x 2 x 128, run to equilibrium
    "coexistence": dict(workload="flat_interface_128", overrides=dict(nx=2, ny=2, nz=128), steps=20000),
    # isothermal static droplet R = 12 in a 40^3 box (stationary after ~2000 steps)
    "laplace": dict(workload="static_droplet_32", overrides=dict(nx=40, ny=40, nz=40, radius=12.0, thermal=0),
                    steps=2000),
    # D^2 test with the reservoir boundary, 32^3, D_0 = 20; D^2 sampled in the
    # quasi-steady window 3000..6000
    "d2": dict(workload="d2_law_48", overrides=dict(nx=32, ny=32, nz=32, radius=10.0), steps=6000, t0=3000,
               every=250),
}


def describe(name):
    """Grid, size and measurement window of a case, for reports."""
    c = CASES[name]
    w = case_workload(name)
    p = w["params"]
    d = {"workload": c["workload"], "grid": [p["nx"], p["ny"], p["nz"]], "steps": c["steps"]}
    if name == "laplace":
        d["radius"] = w["init"]["radius"]
    if name == "d2":
        d.update(D0=2 * w["init"]["radius"], window=[c["t0"], c["steps"]], every=c["every"])
    return d


def case_workload(name):
    c = CASES[name]
    w = copy.deepcopy(W.load(c["workload"]))
    for k, v in c["overrides"].items():
        if k in w["init"]:
            w["init"][k] = v
        else:
            w["params"][k] = v
    return w


def schedule(name):
    """Step counts between readouts and the time of each readout."""
    c = CASES[name]
    if name != "d2":
        return [c["steps"]], [c["steps"]]
    times = list(range(c["t0"], c["steps"] + 1, c["every"]))
    chunks = [times[0]] + [c["every"]] * (len(times) - 1)
    return chunks, times


def slab_densities(rho, p):
    prof = rho.reshape(p["nz"], p["ny"], p["nx"]).mean(axis=(1, 2))
    return float(prof.max()), float(prof.min())


def pressure(rho, T, p):
    """Peng-Robinson pressure of Eq. (49), a = 0.45724 R^2 Tc^2/pc and
    b = 0.0778 R Tc/pc giving Tc = (0.0778/0.45724) a/(b R)."""
    a, b, R, w = p["a"], p["b"], p["R"], p["acentric"]
    Tc = 0.0778 / 0.45724 * a / (b * R)
    kap = 0.37464 + 1.54226 * w - 0.26992 * w * w
    th = (1.0 + kap * (1.0 - np.sqrt(T / Tc))) ** 2
    return rho * R * T / (1.0 - b * rho) - a * th * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho)


def laplace_jump(rho, T, p):
    """p_EOS at the droplet centre minus p_EOS at the box corner."""
    n = rho.reshape(p["nz"], p["ny"], p["nx"])
    t = T.reshape(p["nz"], p["ny"], p["nx"])
    c = (p["nz"] // 2, p["ny"] // 2, p["nx"] // 2)
    pin = pressure(n[c], t[c], p)
    pout = pressure(n[0, 0, 0], t[0, 0, 0], p)
    return float(pin - pout), float(n[c]), float(n[0, 0, 0])


def d2_ratio(rho, w):
    """(D/D_0)^2 with D the diameter of the sphere whose volume is
    sum clip((rho - rho_25)/(rho_75 - rho_25), 0, 1), rho_25 and rho_75 the
    densities a quarter and three quarters of the way from rho_g to rho_l
    (a smooth count of liquid nodes that ignores the slow rise of the vapour
    density)."""
    rl, rg = w["init"]["rho_l"], w["init"]["rho_g"]
    lo, hi = rg + 0.25 * (rl - rg), rg + 0.75 * (rl - rg)
    V = float(np.clip((rho - lo) / (hi - lo), 0.0, 1.0).sum())
    D = 2.0 * (3.0 * V / (4.0 * np.pi)) ** (1.0 / 3.0)
    return (D / (2.0 * w["init"]["radius"])) ** 2


def d2_slope(times, d2):
    return float(np.polyfit(np.asarray(times, float), np.asarray(d2, float), 1)[0])


def run_case(name, make_runner):
    """Run case `name`.  make_runner(w) returns (step(n), read() -> (rho, ux,
    uy, uz, T), close()).  Returns the case's measured numbers."""
    w = case_workload(name)
    p = w["params"]
    step, read, close = make_runner(w)
    chunks, times = schedule(name)
    try:
        if name == "d2":
            d2 = []
            for n in chunks:
                step(n)
                d2.append(d2_ratio(read()[0], w))
            return dict(times=times, d2=d2, slope=d2_slope(times, d2))
        step(chunks[0])
        rho, ux, uy, uz, T = read()
        if name == "coexistence":
            rl, rg = slab_densities(rho, p)
            return dict(rho_l=rl, rho_g=rg)
        dp, rin, rout = laplace_jump(rho, T, p)
        return dict(dp=dp, rho_in=rin, rho_out=rout)
    finally:
        close()


def relative_errors(name, got, ref):
    keys = {"coexistence": ("rho_l", "rho_g"), "laplace": ("dp",), "d2": ("slope",)}[name]
    return {k: abs(got[k] - ref[k]) / abs(ref[k]) for k in keys}
