"""Write tests/golden/precision_refs.json: the coexistence densities, Laplace
jump and D^2 slope of the precision cases (tests/precision_metrics.py)
computed by the FP64 oracle alone.

Run:  python tests/golden/make_precision_refs.py"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import sim  # noqa: E402
from paper_2201_06039_amd import workloads as W  # noqa: E402
import precision_metrics as PM  # noqa: E402


def oracle_runner(w):
    s = sim.Sim(**w["params"])
    s.init_fields(*W.fields(w))
    return s.step, s.rho_u_T, s.close


def main():
    out = {"generated_by": "python tests/golden/make_precision_refs.py (FP64 oracle)", "cases": {}}
    for name in PM.CASES:
        t0 = time.time()
        out["cases"][name] = PM.run_case(name, oracle_runner)
        print(name, {k: v for k, v in out["cases"][name].items() if k not in ("times", "d2")},
              f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, "precision_refs.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
