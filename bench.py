"""Benchmark of the fused D3Q19 + D3Q7 thermal pseudopotential LB step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--storage f16|f32|f64|bf16|f32dev] [--compare f32|none]
                    [--thermal-lattice d3q7|d3q19] [--divu local|fd] [--tile TXxTY] [--chunk CZ]
                    [--no-precision] [--no-d2-full-size] [--no-batch] [--no-lattice-comparison]
                    [--no-workloads] [--workloads NAME,...] [--no-cpu-baseline]

One step = one fused time step of the whole grid (both lattices, streaming and
boundary rules) on synthetic seeded input already resident in HBM.  The
headline workload is the precision form of the method: a 512^3 periodic
field of 64 droplets at T_sat (Sec. IV A parameters) with FP16 deviation
storage, against the same grid with FP32 population storage.  Prints one
JSON line: MLUPS (million lattice-node updates per second) of the chosen
storage, the HBM roofline of the step kernel at the method's algorithmic
bytes per update, the FP32-storage comparison, the errors of the storage
format against the FP64 oracle (coexistence densities, Laplace jump, D^2
slope, each case labelled with its grid and window, and the D^2 test at the
paper's 100^3 size), the batched step over 256 independent lattices of uneven
size, the D3Q19-vs-D3Q7 temperature lattice and finite-difference-vs-Eq. (48)
comparisons and the 128^3 and pool-boiling rates, a streaming-copy ceiling,
and the FP64 oracle timed on the host cores as a CPU baseline.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D3Q19+D3Q7 fused step) + % HBM peak, FP16-store vs FP32 at stated error"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per lattice update: the state the method must move, each
# value read once and written once -- 19 + 7 populations and the phi_s
# history of Eq. (23) (FP32; FP64 for f64).  FP16/BF16 populations: 112 B;
# FP32: 216 B (FP32 deviations move FP32 populations too).
BYTES_ALG = {"f32": 2 * 26 * 4 + 8, "f64": 2 * 26 * 8 + 16, "f16": 2 * 26 * 2 + 8, "bf16": 2 * 26 * 2 + 8,
             "f32dev": 2 * 26 * 4 + 8}
# What the deviation formats move in addition: the per-node references
# rho_r, T_r (FP16 for f16, FP32 for bf16 and f32dev), read and written.
BYTES_WITH_REFERENCES = {"f32": 216, "f64": 432, "f16": 120, "bf16": 128, "f32dev": 232}
# The same with a D3Q19 temperature lattice (19 + 19 populations).
BYTES_ALG_Q19T = {"f32": 2 * 38 * 4 + 8, "f64": 2 * 38 * 8 + 16, "f16": 2 * 38 * 2 + 8}


def bytes_alg(storage, q19t=False):
    return (BYTES_ALG_Q19T if q19t else BYTES_ALG)[storage]


PRECISION_BOUND = 1e-3
# Device code of the step kernels: counter figures stay valid while it is unchanged.
KERNEL_SOURCES = ["paper_2201_06039_amd/csrc/lbm_kernels.hpp"]


def traffic_file(workload, storage, q19t=False):
    tag = "_d3q19t" if q19t else ""
    return os.path.join(ROOT, "profiles", f"k_step_{workload}_{storage}{tag}_traffic.json")


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, storage, launch, q19t=False):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source with the same workload and launch."""
    try:
        with open(traffic_file(workload, storage, q19t)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("workload") != workload or t.get("storage") != storage:
        return None
    if t.get("launch") != [launch["tile_x"], launch["tile_y"], launch["chunk_z"]]:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(p, fields, nz, steps, threads):
    """MLUPS of the FP64 oracle over `steps` steps of the z-slab [0, nz) of a
    field (a box of its own with the workload's boundaries), with `threads`
    OpenMP threads (None: all it is given)."""
    from oracle import sim
    nz = min(nz, p["nz"])
    sl = [f[:nz] for f in fields]
    if threads:
        sim.set_threads(threads)
    s = sim.Sim(**dict(p, nz=nz))
    s.init_fields(*sl)
    t0 = time.perf_counter()
    s.step(steps)
    t1 = time.perf_counter()
    used = sim.max_threads()
    s.close()
    if threads:
        sim.set_threads(0)
    whole = nz == p["nz"]
    return dict(value=round(s.nn * steps / (t1 - t0) / 1e6, 3), cores=used,
                sample=f"{steps} step(s) of the " + (f"{p['nx']}x{p['ny']}x{nz} grid" if whole else
                                                     f"{p['nx']}x{p['ny']}x{nz} slab z < {nz} of the "
                                                     f"{p['nx']}x{p['ny']}x{p['nz']} field")
                       + f", FP64 C + OpenMP, {used} thread(s)")


# Bounded oracle samples of the other workloads: (name, (slab, steps) on all
# threads, (slab, steps) on one thread), about a second each.
CPU_CONFIG_SAMPLES = (("static_droplet_32", (32, 300), (32, 30)),
                      ("evaporation_128", (128, 10), (128, 1)),
                      ("pool_boiling_256x256x384", (64, 2), (16, 1)))


def cpu_baseline(w, fields, slab_all=64, slab_one=8, configs=True):
    """The FP64 oracle (as it stands) on the host cores, on bounded samples of
    the same workload: 2 steps of the z-slab [0, slab_all) of the grid with
    every thread OpenMP gives it, and 1 step of the slab [0, slab_one) on one
    thread.  Each slab is a box of its own (the per-node work of the oracle
    does not depend on the data).  `configs` adds the same pair of figures for
    the smaller workloads (the static droplet, the 128^3 evaporation, the pool
    grid)."""
    from paper_2201_06039_amd import workloads as W
    p = dict(w["params"])
    full = _oracle_rate(p, fields, slab_all, 2, None)
    one = _oracle_rate(p, fields, slab_one, 1, 1)
    out = {"value": full["value"], "unit": "MLUPS", "cores": full["cores"], "kind": "oracle",
           "sample": full["sample"], "single_thread": one, "cpu_model": cpu_model()}
    if configs:
        rows = []
        for name, (nz_all, st_all), (nz_one, st_one) in CPU_CONFIG_SAMPLES:
            wc = W.load(name)
            fc = W.fields(wc)
            pc = dict(wc["params"])
            rows.append({"workload": name, "grid": [pc["nx"], pc["ny"], pc["nz"]],
                         "all_threads": _oracle_rate(pc, fc, nz_all, st_all, None),
                         "single_thread": _oracle_rate(pc, fc, nz_one, st_one, 1)})
        out["configs"] = rows
    return out


def new_stream():
    import torch
    return torch.cuda.Stream(device="cuda:0")  # default priority


def timed_run(lbm, p, fields, storage, steps, warmup, tile=None, chunk=None, repeats=1):
    """Warm up, then time `steps` steps with HIP events on the library's stream
    (its own stream, so pairs of steps replay a captured graph).  With
    repeats > 1 the K-step timing is repeated and every repetition kept; the
    first is the reported one."""
    import torch
    lat = lbm.Lattice(p, storage=storage, device="cuda:0", stream=new_stream())
    if tile or chunk:
        cur = lat.launch()
        tx, ty = (int(v) for v in tile.split("x")) if tile else (cur["tile_x"], cur["tile_y"])
        lat.set_launch(tx, ty, chunk or cur["chunk_z"])
    launch = lat.launch()
    lat.init_fields(*fields)
    lat.step(warmup)
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(lat.stream)
        lat.step(steps)
        end.record(lat.stream)
        torch.cuda.synchronize()
        times.append(start.elapsed_time(end))
    lat.rho_u_T()  # raises if any step was unstable
    launches = lat.launches_per_step()
    lat.close()
    return times[0], launch, launches, times


def copy_ceiling(lbm, mbytes=2048, calls=20):
    """GB/s of the library's streaming copy kernel on `mbytes` MB (read + write)."""
    import torch
    n = mbytes * (1 << 20)
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    lbm.copy_probe(a, b)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(calls):
        lbm.copy_probe(a, b)
    end.record()
    torch.cuda.synchronize()
    sec = start.elapsed_time(end) / 1e3 / calls
    return {"kernel": "k_copy16", "bytes_per_call": 2 * n, "GBps": round(2 * n / sec / 1e9, 1),
            "frac_of_peak": round(2 * n / sec / 1e9 / HBM_PEAK_GBS, 4)}


def precision_errors(storage):
    """Relative errors of the coexistence densities, Laplace jump and D^2
    slope of a run with this storage against the FP64 oracle's values
    (stored in tests/golden/precision_refs.json by the oracle), with each
    case's grid and window."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import precision_metrics as PM
    from paper_2201_06039_amd import lbm, workloads as W
    with open(os.path.join(ROOT, "tests", "golden", "precision_refs.json")) as fh:
        refs = json.load(fh)["cases"]

    def make(w):
        lat = lbm.Lattice(w["params"], storage=storage, device="cuda:0")
        lat.init_fields(*W.fields(w))
        return lat.step, lat.rho_u_T, lat.close

    out = {}
    for case in PM.CASES:
        errs = {k: float(f"{v:.3e}") for k, v in PM.relative_errors(case, PM.run_case(case, make), refs[case]).items()}
        out[case] = {"case": PM.describe(case), "relative_errors": errs,
                     "within_bound": max(errs.values()) <= PRECISION_BOUND}
    return out


def d2_full_size(lbm, W, storages, steps=60000, every=1000):
    """The D^2 test at the size the paper states (Sec. IV A: 100^3, D_0 = 50):
    (D/D_0)^2 read out every `every` steps, and the relative error of its
    slope in each window against the FP64 oracle's run
    (tests/golden/d2_full_oracle.json, windows it reached) -- or, where the
    oracle's run does not reach a window, against the FP64 kernel, which
    matches the oracle to 1e-12 per step (the reference is named per window)."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import precision_metrics as PM
    w = W.load("d2_law_100")
    fields = W.fields(w)
    times = np.arange(every, steps + 1, every)
    ref_path = os.path.join(ROOT, "tests", "golden", "d2_full_oracle.json")
    oracle = None
    if os.path.exists(ref_path):
        with open(ref_path) as fh:
            ref = json.load(fh)
        if ref.get("every") == every and ref["times"] == [int(t) for t in times[:len(ref["times"])]]:
            oracle = np.array(ref["d2"])
    windows = [(w0, w1) for w0, w1 in ((5000, 10000), (10000, 20000), (20000, 40000), (40000, 60000)) if w1 <= steps]
    need_f64 = oracle is None or len(oracle) < len(times)
    runs = list(storages) + (["f64"] if need_f64 and "f64" not in storages else [])
    curves = {}
    for storage in runs:
        lat = lbm.Lattice(w["params"], storage=storage, device="cuda:0", stream=new_stream())
        lat.init_fields(*fields)
        d2 = []
        for _ in times:
            lat.step(every)
            d2.append(PM.d2_ratio(lat.rho_u_T()[0], w))
        lat.close()
        curves[storage] = np.array(d2)
        print(f"# d2 100^3 {storage}: d2(end) = {d2[-1]:.5f}", file=sys.stderr, flush=True)
    out = {"workload": "d2_law_100", "grid": [100, 100, 100], "D0": 50, "steps": steps, "every": every,
           "windows": {}, "d2_end": {k: round(float(c[-1]), 6) for k, c in curves.items()}}
    for w0, w1 in windows:
        sel = (times >= w0) & (times <= w1)
        idx = np.nonzero(sel)[0]
        if oracle is not None and len(oracle) > idx[-1]:
            base, ref_curve = "FP64 oracle", oracle[idx]
        else:
            base, ref_curve = "FP64 kernel", curves["f64"][sel]
        ref_slope = np.polyfit(times[sel], ref_curve, 1)[0]
        errs = {name: round(float((np.polyfit(times[sel], c[sel], 1)[0] - ref_slope) / abs(ref_slope)), 5)
                for name, c in curves.items() if name in storages}
        out["windows"][f"{w0}-{w1}"] = {"reference": base, "slope_relative_error": errs,
                                       "within_bound": {k: abs(v) <= PRECISION_BOUND for k, v in errs.items()}}
    return out


def bubble_departure(lbm, W, name, g=None, storage="f32", max_steps=30000, every=100):
    """Sec. IV C: run the closed-box nucleation workload until a vapour bubble
    leaves the hydrophobic square.  Every `every` steps the vapour nodes
    (rho below the mid-density of the saturated phases) are split into
    connected components; the first component that touches neither the wall
    (z = 0) nor the vapour above the pool is the departed bubble, and its
    equivalent-sphere diameter (6 V / pi)^(1/3) is D_d."""
    import numpy as np
    from scipy import ndimage
    w = W.load(name)
    p = dict(w["params"])
    if g is not None:
        p["grav"] = [0.0, 0.0, -g]
    mid = 0.5 * (w["init"]["rho_l"] + w["init"]["rho_g"])
    lat = lbm.Lattice(p, storage=storage, device="cuda:0", stream=new_stream())
    lat.init_fields(*W.fields(w))
    t0 = time.perf_counter()
    out = {"workload": name, "g": -p["grav"][2], "storage": storage, "departure_step": None, "D_d": None,
           "attached_max_D": 0.0, "readout_every": every}
    t = 0
    while t < max_steps:
        lat.step(every)
        t += every
        rho = lat.rho_u_T()[0]
        lab, n = ndimage.label(rho < mid)
        if n == 0:
            continue
        ids = np.arange(1, n + 1)
        vol = ndimage.sum_labels(np.ones_like(rho), lab, ids)
        zmin = ndimage.minimum(np.broadcast_to(np.arange(p["nz"])[:, None, None], rho.shape), lab, ids)
        zmax = ndimage.maximum(np.broadcast_to(np.arange(p["nz"])[:, None, None], rho.shape), lab, ids)
        attached = [(v, i) for v, i, z0 in zip(vol, ids, zmin) if z0 == 0]
        if attached:
            out["attached_max_D"] = max(out["attached_max_D"], round(float((6 * max(attached)[0] / np.pi) ** (1 / 3)), 2))
        free = [(v, i) for v, i, z0, z1 in zip(vol, ids, zmin, zmax) if z0 > 0 and z1 < p["nz"] - 1 and v > 1000]
        if free:
            v = max(free)[0]
            out.update(departure_step=t, D_d=round(float((6 * v / np.pi) ** (1 / 3)), 2))
            break
    lat.close()
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    print(f"# departure {name}: {out}", file=sys.stderr, flush=True)
    return out


def nucleation_study(lbm, W, name="nucleation_200x200x280", gravities=(1e-5, 1.5e-5, 2e-5, 3e-5, 4e-5)):
    """Departure diameters over a range of gravities and the exponent of
    D_d ~ g^n from a least-squares fit of log D_d against log g (the paper's
    correlation line is D_d = 0.253 g^-0.5, Fig. 7)."""
    import numpy as np
    runs = [bubble_departure(lbm, W, name, g=g) for g in gravities]
    ok = [r for r in runs if r["D_d"]]
    for r in runs:
        r["D_d_correlation"] = round(0.253 * r["g"] ** -0.5, 2)
    out = {"runs": runs, "paper_correlation": "D_d = 0.253 g^-0.5"}
    if len(ok) >= 2:
        slope, icpt = np.polyfit(np.log([r["g"] for r in ok]), np.log([r["D_d"] for r in ok]), 1)
        out.update(exponent=round(float(slope), 3), prefactor=round(float(np.exp(icpt)), 4))
    return out


def ccr_evaporation(lbm, W, name="ccr_evaporation_200x200x100", storage="f32", settle=10000, max_steps=600000,
                    every=5000, stop_fraction=0.25):
    """Sec. IV B: the hemisphere on the heated wall.  The first `settle` steps
    hold the temperature lattice (thermal = 0); the state then continues with
    it (checkpoint into a lattice with thermal = 1).  Every `every` steps:
    the droplet mass (sum of rho over the liquid nodes, rho above the mid
    density), the footprint diameter D = 2 (A/pi)^(1/2) of the liquid nodes of
    the first layer, the apex height h (liquid nodes of the centre column,
    the wall plane at z = -1/2) and the spherical-cap contact angle
    2 atan(2h/D).  Stops when the mass falls below `stop_fraction` of its
    value when heating starts."""
    import numpy as np
    w = W.load(name)
    p = dict(w["params"])
    mid = 0.5 * (w["init"]["rho_l"] + w["init"]["rho_g"])
    cx, cy = (p["nx"] - 1) // 2, (p["ny"] - 1) // 2
    t0 = time.perf_counter()
    lat = lbm.Lattice(dict(p, thermal=0), storage=storage, device="cuda:0", stream=new_stream())
    lat.init_fields(*W.fields(w))
    lat.step(settle)
    blob = lat.get_state()
    lat.close()
    lat = lbm.Lattice(p, storage=storage, device="cuda:0", stream=new_stream())
    lat.set_state(blob)

    def sample(t):
        rho = lat.rho_u_T()[0]
        liq = rho > mid
        area = float(liq[0].sum())
        D = 2.0 * (area / np.pi) ** 0.5
        h = float(liq[:, cy:cy + 2, cx:cx + 2].sum(axis=0).max())
        theta = float(np.degrees(2.0 * np.arctan2(2.0 * h, D))) if D > 0 else 0.0
        return dict(t=t, mass=float(rho[liq].sum()), D=round(D, 2), h=h, theta=round(theta, 1))

    samples = [sample(0)]
    m0 = samples[0]["mass"]
    t = 0
    while t < max_steps and samples[-1]["mass"] > stop_fraction * m0:
        lat.step(every)
        t += every
        samples.append(sample(t))
        q = samples[-1]
        print(f"# ccr {storage} t={t}: mass {q['mass'] / m0:.4f} D {q['D']} h {q['h']} theta {q['theta']}",
              file=sys.stderr, flush=True)
    lat.close()
    for s in samples:
        s["mass"] = round(s["mass"] / m0, 4)
    D0 = samples[0]["D"]
    pinned = [s for s in samples if abs(s["D"] - D0) <= 2.0]
    last_pinned = max((k for k, s in enumerate(samples) if all(abs(q["D"] - D0) <= 2.0 for q in samples[:k + 1])),
                      default=0)
    out = {"workload": name, "storage": storage, "settle_steps": settle, "readout_every": every,
           "D_at_heating": D0, "theta_at_heating": samples[0]["theta"],
           "ccr_until_step": samples[last_pinned]["t"], "mass_at_ccr_end": samples[last_pinned]["mass"],
           "theta_at_ccr_end": samples[last_pinned]["theta"], "samples_with_D_within_2": len(pinned),
           "samples": samples, "wall_s": round(time.perf_counter() - t0, 1)}
    print(f"# ccr {name} {storage}: D {D0} theta {samples[0]['theta']} -> CCR until t = {out['ccr_until_step']} "
          f"(mass {out['mass_at_ccr_end']}, theta {out['theta_at_ccr_end']}); {len(samples)} readouts",
          file=sys.stderr, flush=True)
    return out


def batch_run(storage, steps, warmup, name="batch_256", launch=None):
    """The batched step over the lattices of workload `name`: autotune the
    launch on the initial state (or take `launch` = (tile_x, tile_y, chunk_z,
    workgroups)), then time `steps` steps (graph replays)."""
    import torch
    from paper_2201_06039_amd import lbm, workloads as W
    wb = W.load(name)
    cases = wb["cases"]
    b = lbm.Batch([c["params"] for c in cases], storage=storage, device="cuda:0", stream=new_stream())
    for i, c in enumerate(cases):
        b.init_case(i, *W.fields(c))
    if launch:
        b.set_launch(*launch)
        tuned_ms = None
    else:
        tuned_ms = round(b.autotune(steps=5), 5)
    launch = b.launch()
    tiles = [b.case_tile(i) for i in range(len(cases))]
    b.step(warmup)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    b.step(steps)
    end.record(b.stream)
    end.synchronize()
    ms = start.elapsed_time(end) / steps
    for i in range(len(cases)):
        b.reduce(i)  # raises if any lattice went unstable
    b.close()
    nodes = wb["nodes"]
    slots = sum(-(-c["params"]["nx"] // tx) * -(-c["params"]["ny"] // ty) * thr * c["params"]["nz"]
                for c, (tx, ty, thr) in zip(cases, tiles))
    return {"workload": name, "cases": len(cases), "nodes": nodes, "storage": storage,
            "value": round(nodes / ms / 1e3, 2), "unit": "MLUPS", "ms_per_step": round(ms, 5), "steps": steps,
            "roofline_frac": round(bytes_alg(storage) * nodes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_lup": bytes_alg(storage), "launch": launch, "autotune_ms_per_step": tuned_ms,
            "thread_slot_efficiency": round(nodes / slots, 4), "graph": True}


def rate_row(nn, ms, steps, storage, launch, launches, q19t=False):
    sec = ms / 1e3 / steps
    return {"MLUPS": round(nn / sec / 1e6, 2), "ms_per_step": round(ms / steps, 5),
            "roofline_frac": round(bytes_alg(storage, q19t) * nn / sec / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_lup": bytes_alg(storage, q19t), "launches_per_step": launches,
            "tile": [launch["tile_x"], launch["tile_y"]], "chunk_z": launch["chunk_z"]}


def other_workloads(lbm, W, names, steps, warmup, storages=("f16", "f32")):
    """MLUPS and roofline fraction of the step on further workloads (the
    pool-boiling wall grid adds the rho_ave reduction launch, which the
    fraction counts, and the 128^3 evaporation grid fits the 256 MB
    Infinity Cache in FP16)."""
    out = {}
    for name in names:
        w = W.load(name)
        fields = W.fields(w)
        p = w["params"]
        nn = p["nx"] * p["ny"] * p["nz"]
        row = {"grid": [p["nx"], p["ny"], p["nz"]]}
        for storage in storages:
            ms, launch, launches, _ = timed_run(lbm, p, fields, storage, steps, warmup)
            row[storage] = rate_row(nn, ms, steps, storage, launch, launches)
            print(f"# {name} {storage}: {ms / steps:.5f} ms/step", file=sys.stderr, flush=True)
        out[name] = row
    return out


def lattice_comparison(lbm, p, fields, steps, warmup, storages=("f16", "f32")):
    """The step with the D3Q7 and the D3Q19 temperature lattice, both with the
    BGK collision of Eq. (19) (the only one the paper specifies for both), on
    the same workload and storage: measured speed ratio against the ratio of
    algorithmic bytes per update."""
    nn = p["nx"] * p["ny"] * p["nz"]
    out = {}
    for storage in storages:
        row = {}
        for name, extra in (("d3q7", dict(thermal_bgk=1)), ("d3q19", dict(thermal_bgk=1, thermal_lattice=1))):
            ms, launch, launches, _ = timed_run(lbm, dict(p, **extra), fields, storage, steps, warmup)
            row[name] = rate_row(nn, ms, steps, storage, launch, launches, q19t=name == "d3q19")
            print(f"# temperature lattice {name} {storage}: {ms / steps:.5f} ms/step", file=sys.stderr, flush=True)
        row["speedup_of_d3q7"] = round(row["d3q19"]["ms_per_step"] / row["d3q7"]["ms_per_step"], 3)
        row["bytes_ratio"] = round(row["d3q19"]["bytes_per_lup"] / row["d3q7"]["bytes_per_lup"], 3)
        out[storage] = row
    return out


def divergence_comparison(lbm, p, fields, steps, warmup, storages=("f16", "f32")):
    """The step with div u of Eq. (48) at every node against the practice it
    replaces, isotropic finite differences of u(t) at interior nodes, which
    needs u at every node before the step (a velocity pass of the step's
    shape first)."""
    nn = p["nx"] * p["ny"] * p["nz"]
    out = {}
    for storage in storages:
        row = {}
        for name, mode in (("local_eq48", 0), ("finite_difference", 1)):
            ms, launch, launches, _ = timed_run(lbm, dict(p, divu_mode=mode), fields, storage, steps, warmup)
            row[name] = rate_row(nn, ms, steps, storage, launch, launches)
            print(f"# divergence {name} {storage}: {ms / steps:.5f} ms/step", file=sys.stderr, flush=True)
        row["speedup_of_local"] = round(row["finite_difference"]["ms_per_step"] / row["local_eq48"]["ms_per_step"], 3)
        out[storage] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="multi_droplet_512")
    ap.add_argument("--storage", default="f16", choices=sorted(BYTES_ALG))
    ap.add_argument("--compare", default="f32", choices=sorted(BYTES_ALG) + ["none"],
                    help="second storage format timed on the same workload")
    ap.add_argument("--thermal-lattice", default="d3q7", choices=["d3q7", "d3q19"],
                    help="temperature lattice of the timed step (d3q19 runs the BGK collision)")
    ap.add_argument("--tile", default=None, help="TXxTY, e.g. 64x4")
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-d2-full-size", action="store_true", help="skip the 100^3 D^2 windows in the precision leg")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched leg and print its JSON")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-launch", default=None, metavar="TXxTYxCZxWG",
                    help="fixed batch launch (tile, chunk, workgroups) instead of the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lattice-comparison", action="store_true")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other-workload leg")
    ap.add_argument("--no-copy", action="store_true", help="skip the streaming-copy ceiling")
    ap.add_argument("--d2-full", action="store_true",
                    help="only run the D^2 test at 100^3 for 60000 steps in every storage format (about 40 s) "
                         "and print its JSON")
    ap.add_argument("--nucleation", action="store_true",
                    help="only run the bubble nucleation and departure test of Sec. IV C at five gravities "
                         "(a few minutes) and print its JSON")
    ap.add_argument("--ccr", action="store_true",
                    help="only run the evaporation of a pinned droplet on the heated wall of Sec. IV B (every "
                         "storage format, several minutes) and print its JSON")
    ap.add_argument("--workloads", default="evaporation_128,pool_boiling_256x256x384",
                    help="comma-separated workloads timed in the other-workload leg")
    ap.add_argument("--divu", default="local", choices=["local", "fd"],
                    help="velocity divergence of the timed step: Eq. (48) or finite differences")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="only run 21 streaming copies of MB megabytes with the library's copy kernel (to "
                         "calibrate the FETCH_SIZE/WRITE_SIZE counters against a kernel of known traffic) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_06039_amd import lbm, workloads as W

    if args.copy_probe:
        print(json.dumps(dict(copy_ceiling(lbm, args.copy_probe), calls=21)), flush=True)
        return

    if args.d2_full:
        print(json.dumps(d2_full_size(lbm, W, ("f64", "f32", "f32dev", "f16", "bf16"))), flush=True)
        return

    if args.nucleation:
        print(json.dumps(nucleation_study(lbm, W)), flush=True)
        return

    if args.ccr:
        runs = [ccr_evaporation(lbm, W, storage=st) for st in ("f64", "f32", "f32dev", "f16", "bf16")]
        ref = {s["t"]: s for s in runs[0]["samples"]}
        for r in runs[1:]:
            common = [s for s in r["samples"] if s["t"] in ref]
            r["vs_f64"] = {k: round(max(abs(s[k] - ref[s["t"]][k]) for s in common), 4) for k in ("mass", "D", "theta")}
        print(json.dumps({"ccr_evaporation": runs}), flush=True)
        return

    if args.batch_only:
        bl = tuple(int(v) for v in args.batch_launch.split("x")) if args.batch_launch else None
        out = batch_run(args.storage, args.batch_steps, args.warmup, launch=bl)
        print(json.dumps(out), flush=True)
        return

    w = W.load(args.workload)
    t0 = time.perf_counter()
    fields = W.fields(w)
    print(f"# fields of {args.workload}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    p = dict(w["params"])
    q19t = args.thermal_lattice == "d3q19"
    if q19t:
        if args.storage not in BYTES_ALG_Q19T:
            ap.error(f"the D3Q19 temperature lattice is built for {sorted(BYTES_ALG_Q19T)}")
        p.update(thermal_lattice=1, thermal_bgk=1)
    fd = args.divu == "fd"
    if fd:
        p["divu_mode"] = 1
    nn = p["nx"] * p["ny"] * p["nz"]
    extras = not q19t and not fd

    print(f"# workload {args.workload} {p['nx']}x{p['ny']}x{p['nz']} storage {args.storage}", file=sys.stderr,
          flush=True)
    ms, launch, launches, reps = timed_run(lbm, p, fields, args.storage, args.steps, args.warmup, args.tile,
                                           args.chunk, repeats=5)
    print(f"# {args.storage}: {ms / args.steps:.5f} ms/step, launch {launch}, repeats {reps}", file=sys.stderr,
          flush=True)

    sec = ms / 1e3
    mlups = nn * args.steps / sec / 1e6
    # The default grid takes one launch per step (periodic, no gravity,
    # Eq. (48)), so the average step time is the step kernel's average launch
    # duration.  Grids with gravity or a wettable wall add a small reduction
    # or wall kernel to each step; the rate is then taken over the whole step,
    # which slightly understates the step kernel's own.
    avg_launch_s = sec / args.steps
    balg = bytes_alg(args.storage, q19t) * nn
    achieved = balg / avg_launch_s / 1e9
    arith = "f64" if args.storage == "f64" else "f32"
    med = statistics.median(reps) / args.steps
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": arith,
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [p["nx"], p["ny"], p["nz"]], "storage": args.storage,
                   "temperature_lattice": args.thermal_lattice.upper() + (" BGK" if q19t else " MRT"),
                   "velocity_divergence": "finite differences" if fd else "Eq. (48)",
                   "tile": [launch["tile_x"], launch["tile_y"]], "chunk_z": launch["chunk_z"],
                   "workgroups": launch["workgroups"], "launches_per_step": launches,
                   "timing": "HIP events on the library's stream, pairs of steps as graph replays"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload, args.storage, launch, q19t),
                     "kernel": "k_step", "bytes_per_lup": bytes_alg(args.storage, q19t),
                     "frac_with_references": None if q19t else round(
                         BYTES_WITH_REFERENCES[args.storage] * nn / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4),
                     "bytes_per_lup_with_references": None if q19t else BYTES_WITH_REFERENCES[args.storage]},
        "repeats": {"runs": len(reps), "ms_per_step": [round(r / args.steps, 5) for r in reps],
                    "median_ms_per_step": round(med, 5), "median_MLUPS": round(nn / (med / 1e3) / 1e6, 2)},
    }
    if args.compare != "none" and args.compare != args.storage and (not q19t or args.compare in BYTES_ALG_Q19T):
        ms2, launch2, launches2, _ = timed_run(lbm, p, fields, args.compare, args.steps, args.warmup)
        print(f"# {args.compare}: {ms2 / args.steps:.5f} ms/step, launch {launch2}", file=sys.stderr, flush=True)
        row = rate_row(nn, ms2, args.steps, args.compare, launch2, launches2, q19t)
        row.update(storage=args.compare, value=row["MLUPS"], unit="MLUPS", speedup_of_storage=round(ms2 / ms, 3))
        out["compare"] = row
    if not args.no_copy:
        out["copy_ceiling"] = copy_ceiling(lbm)
        print(f"# copy ceiling: {out['copy_ceiling']}", file=sys.stderr, flush=True)
    del fields
    if not args.no_workloads and extras and args.workloads:
        out["workloads"] = other_workloads(lbm, W, args.workloads.split(","), 200, 10)
    if not args.no_lattice_comparison and extras:
        w128 = W.load("evaporation_128")
        f128 = W.fields(w128)
        out["temperature_lattice_comparison"] = dict(
            workload="evaporation_128", **lattice_comparison(lbm, w128["params"], f128, 500, 20))
        out["divergence_comparison"] = dict(
            workload="evaporation_128", **divergence_comparison(lbm, w128["params"], f128, 250, 20))
    if not args.no_precision and extras:
        # the timed storage and the comparison storage, each against the oracle
        stores = [args.storage] + ([args.compare] if args.compare not in ("none", args.storage) else [])
        prec = {"storage": args.storage, "reference": "FP64 oracle", "bound": PRECISION_BOUND}
        d2 = d2_full_size(lbm, W, tuple(stores)) if not args.no_d2_full_size else None
        for st in stores:
            errs = precision_errors(st)
            print(f"# precision of {st}: {errs}", file=sys.stderr, flush=True)
            flags = [c["within_bound"] for c in errs.values()]
            if d2:
                flags += [win["within_bound"][st] for win in d2["windows"].values()]
            key = "cases" if st == args.storage else f"compare_{st}"
            prec[key] = errs
            prec["within_bound" if st == args.storage else f"compare_{st}_within_bound"] = all(flags)
        if d2:
            prec["d2_100"] = d2
        out["precision"] = prec
    if not args.no_batch and extras:
        bl = tuple(int(v) for v in args.batch_launch.split("x")) if args.batch_launch else None
        out["batch"] = batch_run(args.storage if args.storage != "f64" else "f32", args.batch_steps, 10, launch=bl)
        print(f"# batch: {out['batch']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, W.fields(w))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
