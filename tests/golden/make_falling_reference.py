"""Write the FP64 oracle reference of the falling-droplet workload
(256 x 1024, walls all round, R = 32, g = 1e-6, corrected model, 50k steps).

Calls only the oracle and the seeded workload generator.  Output:
tests/golden/falling256x1024_oracle.npz with
  phi_final   float32 [ny, nx]   order parameter at the last step
  t           int64   [K]        diagnostic times (every 1000 steps)
  centroid    float64 [K, 2]     centroid (clamped-phi weights)
  centroid_vel float64 [K, 2]
  second_moment float64 [K, 2]
  mass        float64 [K]
Run: OMP_NUM_THREADS=8 python tests/golden/make_falling_reference.py [steps]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402


def main(steps=50000, every=1000, out=None):
    case = W.falling_droplet()
    s = O.Sim(case.params, case.phi0, case.u0, case.p0)
    rec = dict(t=[], centroid=[], centroid_vel=[], second_moment=[], mass=[])

    def record():
        d = s.diag()
        rec["t"].append(s.time)
        rec["centroid"].append(d["centroid"][:2])
        rec["centroid_vel"].append(d["centroid_vel"][:2])
        rec["second_moment"].append(d["second_moment"][:2])
        rec["mass"].append(d["mass"])

    record()
    t0 = time.time()
    while s.time < steps:
        s.step(min(every, steps - s.time))
        record()
        print(f"t={s.time} centroid={rec['centroid'][-1]} vel={rec['centroid_vel'][-1]} "
              f"wall={time.time() - t0:.0f}s", flush=True)
    fl = s.fields()
    nx, ny = case.params["nx"], case.params["ny"]
    out = out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                              f"falling{nx}x{ny}_oracle.npz")
    np.savez_compressed(out, phi_final=fl["phi"].reshape(ny, nx).astype(np.float32),
                        **{k: np.array(v) for k, v in rec.items()})
    print("wrote", out)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 50000)
