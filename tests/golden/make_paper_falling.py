"""Write the FP64 oracle reference of the paper's falling-droplet test at its
own size (150 x 450, periodic x, D = 32, Eo = 17; `workloads.paper_falling`)
for the original (remove_fa = 0) and the corrected (remove_fa = 1) model,
20k steps each.

Calls only the oracle and the seeded workload generator.  Output:
tests/golden/paper_falling150x450_oracle.npz with, for m in (0, 1):
  t               int64   [K]      diagnostic times (every 500 steps)
  centroid_y_m    float64 [K]      vertical centroid (clamped-phi weights)
  velocity_y_m    float64 [K]      vertical centroid velocity
  spread_m        float64 [K]      spread radius (largest row half-width of
                                   the phi = 1/2 contour, the paper's Fig. 5)
  mass_m          float64 [K]
Run: OMP_NUM_THREADS=8 python tests/golden/make_paper_falling.py [steps]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402


def run(remove_fa, steps, every):
    case = W.paper_falling(remove_fa=remove_fa)
    nx, ny = case.params["nx"], case.params["ny"]
    s = O.Sim(case.params, case.phi0, case.u0, case.p0)
    rec = dict(t=[], cy=[], vy=[], spread=[], mass=[])

    def record():
        d = s.diag()
        rec["t"].append(s.time)
        rec["cy"].append(d["centroid"][1])
        rec["vy"].append(d["centroid_vel"][1])
        rec["spread"].append(O.spread_radius(s.fields()["phi"], (nx, ny)))
        rec["mass"].append(d["mass"])

    record()
    t0 = time.time()
    while s.time < steps:
        s.step(min(every, steps - s.time))
        record()
        print(f"remove_fa={remove_fa} t={s.time} yc={rec['cy'][-1]:.3f} "
              f"spread={rec['spread'][-1]:.3f} wall={time.time() - t0:.0f}s", flush=True)
    return rec


def main(steps=20000, every=500, out=None):
    arrays = {}
    for m in (0, 1):
        rec = run(m, steps, every)
        arrays["t"] = np.array(rec["t"], dtype=np.int64)
        arrays[f"centroid_y_{m}"] = np.array(rec["cy"])
        arrays[f"velocity_y_{m}"] = np.array(rec["vy"])
        arrays[f"spread_{m}"] = np.array(rec["spread"])
        arrays[f"mass_{m}"] = np.array(rec["mass"])
    out = out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                              "paper_falling150x450_oracle.npz")
    np.savez_compressed(out, **arrays)
    print("wrote", out)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 20000)
