"""Write oracle reference trajectories for the full-size workloads.

Calls only the oracle (and the seeded workload definitions).  The GPU
parity tests compare the library against these stored values at the sizes
whose oracle run takes too long to repeat inside a test (the N = 21 chain
with chi <= 64 takes tens of minutes on 8 cores).

    python tests/golden/make_oracle_golden.py xy21 [n_steps]

Output: tests/golden/<name>_oracle.json with <sigma^z_n> (real and imag
parts) at steps 0..n_steps, Tr rho, and the bond dimensions.
"""
import json
import os
import sys
import time
import warnings

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
warnings.filterwarnings("ignore")

import numpy as np  # noqa: E402

from oracle import pt_tebd  # noqa: E402
from oracle.build import problem_from_workload  # noqa: E402
from paper_2201_05529_amd import workloads as W  # noqa: E402


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "xy21"
    wl = getattr(W, name)()
    n_steps = int(sys.argv[2]) if len(sys.argv) > 2 else wl["n_steps"]
    prob, _ = problem_from_workload(wl)
    eng = pt_tebd.Engine(prob)
    n = wl["n_sites"]
    rec = {"workload": name, "n_steps": n_steps, "sz_re": [], "sz_im": [], "trace_re": [], "trace_im": [],
           "chi": [], "seconds": []}
    t0 = time.time()

    def record():
        vals = [eng.expectation(s, W.SZ) for s in range(n)]
        tr = eng.trace()
        rec["sz_re"].append([float(np.real(v)) for v in vals])
        rec["sz_im"].append([float(np.imag(v)) for v in vals])
        rec["trace_re"].append(float(np.real(tr)))
        rec["trace_im"].append(float(np.imag(tr)))
        rec["chi"].append([int(c) for c in eng.mps.bond_dims()])
        rec["seconds"].append(time.time() - t0)

    record()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    for k in range(1, n_steps + 1):
        eng.step(1)
        record()
        print(f"step {k} {time.time() - t0:.1f}s chi={rec['chi'][-1]}", flush=True)
        if k % 5 == 0 or k == n_steps:
            with open(out + ".tmp", "w") as f:
                json.dump(rec, f)
            os.replace(out + ".tmp", out)


if __name__ == "__main__":
    main()
