"""Benchmark of the fused D3Q19 + D3Q7 thermal pseudopotential LB step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--storage f16|f32|f64|bf16|f32dev] [--compare f32|none]
                    [--thermal-lattice d3q7|d3q19] [--divu local|fd] [--tile TXxTY] [--chunk CZ]
                    [--no-precision] [--no-batch] [--no-lattice-comparison] [--no-workloads]
                    [--workloads NAME,...] [--no-cpu-baseline]

One step = one fused time step of the whole grid (both lattices, streaming and
boundary rules) on synthetic seeded input already resident in HBM.  Prints one
JSON line: MLUPS (million lattice-node updates per second) of the chosen
population storage (FP16 deviations by default), the HBM roofline of the step
kernel, the same step with FP32 storage for comparison, the errors of the
storage format against the FP64 oracle's reference values (coexistence
densities, Laplace jump, D^2 slope), the batched step over 256 independent
lattices of uneven size (aggregate MLUPS after autotuning), the same step with
a D3Q19 temperature lattice against the D3Q7 one (the paper's efficiency
argument for D3Q7, Sec. III B), the rates on the pool-boiling wall grid, and
the FP64 oracle timed on the host as a CPU baseline.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D3Q19+D3Q7 fused step) + % HBM peak, FP16-store vs FP32 at stated error"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per lattice update: 19 + 7 populations (plus the two
# reference values rho_r, T_r of the deviation formats: FP16 for f16, FP32
# for bf16 and f32dev) and the FP32 phi_s history (FP64 for f64), each read
# once and written once.
BYTES_PER_LUP = {"f32": 2 * 26 * 4 + 8, "f64": 2 * 26 * 8 + 16, "f16": 2 * (26 * 2 + 2 * 2) + 8,
                 "bf16": 2 * (26 * 2 + 2 * 4) + 8, "f32dev": 2 * 28 * 4 + 8}
# The same with a D3Q19 temperature lattice: 19 + 19 populations.
BYTES_PER_LUP_Q19T = {"f32": 2 * 38 * 4 + 8, "f64": 2 * 38 * 8 + 16, "f16": 2 * (38 * 2 + 2 * 2) + 8}


def bytes_per_lup(storage, q19t=False):
    return (BYTES_PER_LUP_Q19T if q19t else BYTES_PER_LUP)[storage]
PRECISION_BOUND = 1e-3
KERNEL_SOURCES = ["paper_2201_06039_amd/csrc/lbm_kernels.hpp", "paper_2201_06039_amd/csrc/lbm_api.hip"]


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


def cpu_baseline(params, fields, seconds=15.0):
    """The FP64 oracle on the host cores, on the same workload, for a bounded
    number of steps sized to take about `seconds`."""
    from oracle import sim
    s = sim.Sim(**params)
    s.init_fields(*fields)
    t0 = time.perf_counter()
    s.step(1)
    t1 = time.perf_counter()
    per = max(t1 - t0, 1e-3)
    n = max(1, int(seconds / per) - 1)
    t0 = time.perf_counter()
    s.step(n)
    t1 = time.perf_counter()
    nn = s.nn
    s.close()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nn * n / (t1 - t0) / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{n} steps of the full {params['nx']}x{params['ny']}x{params['nz']} grid "
                      f"after 1 untimed step, FP64 C + OpenMP"}


def timed_run(lbm, p, fields, storage, steps, warmup, tile=None, chunk=None):
    """Warm up, then time `steps` steps with HIP events on the library's stream."""
    import torch
    lat = lbm.Lattice(p, storage=storage, device="cuda:0")
    if tile or chunk:
        cur = lat.launch()
        tx, ty = (int(v) for v in tile.split("x")) if tile else (cur["tile_x"], cur["tile_y"])
        lat.set_launch(tx, ty, chunk or cur["chunk_z"])
    launch = lat.launch()
    lat.init_fields(*fields)
    lat.step(warmup)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.step(steps)
    end.record(lat.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    lat.rho_u_T()  # raises if any step was unstable
    launches = lat.launches_per_step()
    lat.close()
    return ms, launch, launches


def precision_errors(storage):
    """Relative errors of the coexistence densities, Laplace jump and D^2
    slope of a run with this storage against the FP64 oracle's values
    (stored in tests/golden/precision_refs.json by the oracle)."""
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
        for k, v in PM.relative_errors(case, PM.run_case(case, make), refs[case]).items():
            out[f"{case}_{k}"] = float(f"{v:.3e}")
    return out


def batch_run(storage, steps, warmup, name="batch_256", launch=None):
    """The batched step over the lattices of workload `name`: autotune the
    launch on the initial state (or take `launch` = (tile_x, tile_y, chunk_z,
    workgroups)), then time `steps` steps (graph replays)."""
    import torch
    from paper_2201_06039_amd import lbm, workloads as W
    wb = W.load(name)
    cases = wb["cases"]
    b = lbm.Batch([c["params"] for c in cases], storage=storage, device="cuda:0")
    for i, c in enumerate(cases):
        b.init_case(i, *W.fields(c))
    if launch:
        b.set_launch(*launch)
        tuned_ms = None
    else:
        tuned_ms = round(b.autotune(steps=5), 5)
    launch = b.launch()
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
    tx, ty = launch["tile_x"], launch["tile_y"]
    slots = sum(-(-c["params"]["nx"] // tx) * tx * -(-c["params"]["ny"] // ty) * ty * c["params"]["nz"] for c in cases)
    return {"workload": name, "cases": len(cases), "nodes": nodes, "storage": storage,
            "value": round(nodes / ms / 1e3, 2), "unit": "MLUPS", "ms_per_step": round(ms, 5), "steps": steps,
            "roofline_frac": round(BYTES_PER_LUP[storage] * nodes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "launch": launch, "autotune_ms_per_step": tuned_ms,
            "thread_slot_efficiency": round(nodes / slots, 4), "graph": True}


def other_workloads(lbm, W, names, steps, warmup, storages=("f16", "f32")):
    """MLUPS and roofline fraction of the step on further workloads (the
    pool-boiling wall grid by default; its step adds the rho_ave reduction
    launch, which the fraction counts)."""
    out = {}
    for name in names:
        w = W.load(name)
        fields = W.fields(w)
        p = w["params"]
        nn = p["nx"] * p["ny"] * p["nz"]
        row = {"grid": [p["nx"], p["ny"], p["nz"]]}
        for storage in storages:
            ms, launch, launches = timed_run(lbm, p, fields, storage, steps, warmup)
            sec = ms / 1e3 / steps
            row[storage] = {"MLUPS": round(nn / sec / 1e6, 2), "ms_per_step": round(ms / steps, 5),
                            "roofline_frac": round(bytes_per_lup(storage) * nn / sec / 1e9 / HBM_PEAK_GBS, 4),
                            "launches_per_step": launches, "tile": [launch["tile_x"], launch["tile_y"]],
                            "chunk_z": launch["chunk_z"]}
            print(f"# {name} {storage}: {ms / steps:.5f} ms/step", file=sys.stderr, flush=True)
        out[name] = row
    return out


def d2_full(lbm, W, storages=("f64", "f32", "f32dev", "f16", "bf16"), steps=60000, every=1000):
    """The D^2 test at the size the paper states (Sec. IV A: 100^3, D_0 = 50)
    for `steps` steps in every storage format: (D/D_0)^2 read out every
    `every` steps, and the slope of each window against that of the FP64
    kernel (and of the FP64 oracle, where tests/golden/d2_full_oracle.json
    holds its values)."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import precision_metrics as PM
    w = W.load("d2_law_100")
    fields = W.fields(w)
    times = np.arange(every, steps + 1, every)
    curves = {}
    for storage in storages:
        lat = lbm.Lattice(w["params"], storage=storage, device="cuda:0")
        lat.init_fields(*fields)
        d2 = []
        for _ in times:
            lat.step(every)
            d2.append(PM.d2_ratio(lat.rho_u_T()[0], w))
        lat.close()
        curves[storage] = np.array(d2)
        print(f"# d2_full {storage}: d2(end) = {d2[-1]:.5f}", file=sys.stderr, flush=True)
    ref_path = os.path.join(ROOT, "tests", "golden", "d2_full_oracle.json")
    if os.path.exists(ref_path):
        with open(ref_path) as fh:
            ref = json.load(fh)
        if ref["times"] == [int(t) for t in times]:
            curves["oracle"] = np.array(ref["d2"])
    windows = [(w0, w1) for w0, w1 in ((5000, 10000), (10000, 20000), (20000, 40000), (40000, 60000)) if w1 <= steps]
    out = {"workload": "d2_law_100", "steps": steps, "every": every, "slope_relative_error": {}, "d2_end": {}}
    for name, c in curves.items():
        out["d2_end"][name] = round(float(c[-1]), 6)
    base = "oracle" if "oracle" in curves else "f64"
    out["reference"] = base
    for w0, w1 in windows:
        sel = (times >= w0) & (times <= w1)
        ref_slope = np.polyfit(times[sel], curves[base][sel], 1)[0]
        out["slope_relative_error"][f"{w0}-{w1}"] = {
            name: round(float((np.polyfit(times[sel], c[sel], 1)[0] - ref_slope) / abs(ref_slope)), 5)
            for name, c in curves.items() if name != base}
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
            ms, launch, _ = timed_run(lbm, dict(p, **extra), fields, storage, steps, warmup)
            row[name] = {"MLUPS": round(nn * steps / (ms / 1e3) / 1e6, 2), "ms_per_step": round(ms / steps, 5),
                         "bytes_per_lup": bytes_per_lup(storage, name == "d3q19"),
                         "tile": [launch["tile_x"], launch["tile_y"]], "chunk_z": launch["chunk_z"]}
            print(f"# temperature lattice {name} {storage}: {ms / steps:.5f} ms/step", file=sys.stderr, flush=True)
        row["speedup_of_d3q7"] = round(row["d3q19"]["ms_per_step"] / row["d3q7"]["ms_per_step"], 3)
        row["bytes_ratio"] = round(row["d3q19"]["bytes_per_lup"] / row["d3q7"]["bytes_per_lup"], 3)
        out[storage] = row
    return out


def divergence_comparison(lbm, p, fields, steps, warmup, storages=("f16", "f32")):
    """The step with div u of Eq. (48) at every node against the practice it
    replaces, isotropic finite differences of u(t) at interior nodes, which
    needs u at every node before the step (here two more passes over the
    state, into FP64 staging planes)."""
    nn = p["nx"] * p["ny"] * p["nz"]
    out = {}
    for storage in storages:
        row = {}
        for name, mode in (("local_eq48", 0), ("finite_difference", 1)):
            ms, launch, launches = timed_run(lbm, dict(p, divu_mode=mode), fields, storage, steps, warmup)
            row[name] = {"MLUPS": round(nn * steps / (ms / 1e3) / 1e6, 2), "ms_per_step": round(ms / steps, 5),
                         "launches_per_step": launches, "tile": [launch["tile_x"], launch["tile_y"]],
                         "chunk_z": launch["chunk_z"]}
            print(f"# divergence {name} {storage}: {ms / steps:.5f} ms/step", file=sys.stderr, flush=True)
        row["speedup_of_local"] = round(row["finite_difference"]["ms_per_step"] / row["local_eq48"]["ms_per_step"], 3)
        out[storage] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="evaporation_128")
    ap.add_argument("--storage", default="f16", choices=sorted(BYTES_PER_LUP))
    ap.add_argument("--compare", default="f32", choices=sorted(BYTES_PER_LUP) + ["none"],
                    help="second storage format timed on the same workload")
    ap.add_argument("--thermal-lattice", default="d3q7", choices=["d3q7", "d3q19"],
                    help="temperature lattice of the timed step (d3q19 runs the BGK collision)")
    ap.add_argument("--tile", default=None, help="TXxTY, e.g. 64x4")
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched leg and print its JSON")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-launch", default=None, metavar="TXxTYxCZxWG",
                    help="fixed batch launch (tile, chunk, workgroups) instead of the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lattice-comparison", action="store_true")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other-workload leg")
    ap.add_argument("--d2-full", action="store_true",
                    help="only run the D^2 test at 100^3 for 60000 steps in every storage format (about 40 s) "
                         "and print its JSON")
    ap.add_argument("--workloads", default="pool_boiling_256x256x384",
                    help="comma-separated workloads timed in the other-workload leg")
    ap.add_argument("--divu", default="local", choices=["local", "fd"],
                    help="velocity divergence of the timed step: Eq. (48) or finite differences")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="only run 20 plain device-to-device copies of MB megabytes (to calibrate the "
                         "FETCH_SIZE/WRITE_SIZE counters against a kernel of known traffic) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(20):
            b.copy_(a)
        end.record()
        torch.cuda.synchronize()
        sec = start.elapsed_time(end) / 1e3 / 20
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "calls": 21,
                          "copy_probe_GBps": round(8 * n / sec / 1e9, 1)}))
        return

    from paper_2201_06039_amd import lbm, workloads as W

    if args.d2_full:
        print(json.dumps(d2_full(lbm, W)), flush=True)
        return

    if args.batch_only:
        bl = tuple(int(v) for v in args.batch_launch.split("x")) if args.batch_launch else None
        out = batch_run(args.storage, args.batch_steps, args.warmup, launch=bl)
        print(json.dumps(out), flush=True)
        return

    w = W.load(args.workload)
    fields = W.fields(w)
    p = dict(w["params"])
    q19t = args.thermal_lattice == "d3q19"
    if q19t:
        if args.storage not in BYTES_PER_LUP_Q19T:
            ap.error(f"the D3Q19 temperature lattice is built for {sorted(BYTES_PER_LUP_Q19T)}")
        p.update(thermal_lattice=1, thermal_bgk=1)
    fd = args.divu == "fd"
    if fd:
        p["divu_mode"] = 1
    nn = p["nx"] * p["ny"] * p["nz"]

    print(f"# workload {args.workload} {p['nx']}x{p['ny']}x{p['nz']} storage {args.storage}", file=sys.stderr,
          flush=True)
    ms, launch, launches = timed_run(lbm, p, fields, args.storage, args.steps, args.warmup, args.tile, args.chunk)
    print(f"# {args.storage}: {ms / args.steps:.5f} ms/step, launch {launch}", file=sys.stderr, flush=True)

    sec = ms / 1e3
    mlups = nn * args.steps / sec / 1e6
    avg_launch_s = sec / args.steps  # the step kernel is the only launch per step when launches == 1
    bytes_alg = bytes_per_lup(args.storage, q19t) * nn
    achieved = bytes_alg / avg_launch_s / 1e9
    arith = "f64" if args.storage == "f64" else "f32"
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
                   "workgroups": launch["workgroups"], "launches_per_step": launches},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload, args.storage, launch, q19t),
                     "kernel": "k_step", "bytes_per_lup": bytes_per_lup(args.storage, q19t)},
    }
    if args.compare != "none" and args.compare != args.storage and (not q19t or args.compare in BYTES_PER_LUP_Q19T):
        ms2, launch2, _ = timed_run(lbm, p, fields, args.compare, args.steps, args.warmup)
        print(f"# {args.compare}: {ms2 / args.steps:.5f} ms/step, launch {launch2}", file=sys.stderr, flush=True)
        sec2 = ms2 / 1e3 / args.steps
        out["compare"] = {"storage": args.compare, "value": round(nn / sec2 / 1e6, 2), "unit": "MLUPS",
                          "ms_per_step": round(ms2 / args.steps, 5),
                          "roofline_frac": round(bytes_per_lup(args.compare, q19t) * nn / sec2 / 1e9 / HBM_PEAK_GBS, 4),
                          "bytes_per_lup": bytes_per_lup(args.compare, q19t),
                          "tile": [launch2["tile_x"], launch2["tile_y"]], "chunk_z": launch2["chunk_z"],
                          "speedup_of_storage": round(ms2 / ms, 3)}
    if not args.no_lattice_comparison and not q19t and not fd:
        out["temperature_lattice_comparison"] = lattice_comparison(lbm, p, fields, max(1, args.steps // 2),
                                                                   args.warmup)
        out["divergence_comparison"] = divergence_comparison(lbm, p, fields, max(1, args.steps // 4), args.warmup)
    if not args.no_workloads and not q19t and not fd and args.workloads:
        out["workloads"] = other_workloads(lbm, W, args.workloads.split(","), 200, 10)
    if not args.no_precision and not q19t and not fd:
        errs = precision_errors(args.storage)
        print(f"# precision of {args.storage}: {errs}", file=sys.stderr, flush=True)
        out["precision"] = {"storage": args.storage, "reference": "FP64 oracle", "bound": PRECISION_BOUND,
                            "relative_errors": errs, "within_bound": max(errs.values()) <= PRECISION_BOUND}
    if not args.no_batch and not q19t and not fd:
        bl = tuple(int(v) for v in args.batch_launch.split("x")) if args.batch_launch else None
        out["batch"] = batch_run(args.storage if args.storage != "f64" else "f32", args.batch_steps, 10, launch=bl)
        print(f"# batch: {out['batch']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, fields)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
