"""Write tests/golden/d2_full_oracle.json: the FP64 oracle's (D/D_0)^2 of the
D^2 test at the size the paper states it (Sec. IV A: a 100^3 box, D_0 = 50,
vapour 0.14 Tc above saturation, constant-temperature boundary), read out
every 1000 steps up to 60000.  Runs the oracle only (about 4.5 h on 8 cores).
The file is rewritten after every readout ("complete": false until the last
one), so an interrupted run leaves the readouts it reached.

    python tests/golden/make_d2_full_ref.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

STEPS, EVERY = 60000, 1000


def main():
    from oracle import sim
    from paper_2201_06039_amd import workloads as W
    import precision_metrics as PM
    w = W.load("d2_law_100")
    s = sim.Sim(**w["params"])
    s.init_fields(*W.fields(w))
    times, d2 = [], []
    t0 = time.time()
    for t in range(EVERY, STEPS + 1, EVERY):
        s.step(EVERY)
        times.append(t)
        d2.append(PM.d2_ratio(s.rho_u_T()[0], w))
        print(f"t={t} d2={d2[-1]:.6f} ({time.time() - t0:.0f} s)", flush=True)
        out = {"workload": "d2_law_100", "steps": STEPS, "every": EVERY, "times": times, "d2": d2,
               "complete": t == STEPS, "generated_by": "python tests/golden/make_d2_full_ref.py (FP64 oracle)"}
        tmp = os.path.join(HERE, "d2_full_oracle.json.tmp")
        with open(tmp, "w") as fh:
            json.dump(out, fh, indent=1)
        os.replace(tmp, os.path.join(HERE, "d2_full_oracle.json"))


if __name__ == "__main__":
    main()
