"""Write oracle reference trajectories for the full-size workloads.

Calls only the oracle (and the seeded workload definitions).  The GPU
parity tests compare the library against these stored values at the sizes
whose oracle run takes too long to repeat inside a test (the N = 21 chain
with chi <= 64 takes about 100 minutes on 8 cores for its 100 steps).

    python tests/golden/make_oracle_golden.py xy21 [n_steps]
    python tests/golden/make_oracle_golden.py xy21 [n_steps] --spread

The first form writes tests/golden/<name>_oracle.json: <sigma^z_n> (real and
imaginary parts) at steps 0..n_steps, Tr rho and the bond dimensions.

The second form writes tests/golden/<name>_spread.json: how far the
oracle's own trajectory moves, step by step, under changes that any other
correct double-precision implementation makes as well:
  * every entry of every site tensor multiplied by (1 + 1e-15 z), z complex
    normal, after every step (two seeds): rounding-level perturbations;
  * every SVD computed by LAPACK's gesvd (QR iteration) instead of gesdd
    (divide and conquer): a second LAPACK implementation of the same steps.
For each step it stores the largest deviation from the unperturbed run over
all <sigma^z_n> and over Tr rho, per variant and as the maximum.
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


def trajectory(prob, n, n_steps, perturb_seed=None, driver="gesdd", rel=1e-15, log=None):
    """<sigma^z_n> for every site and Tr rho at steps 0..n_steps."""
    eng = pt_tebd.Engine(prob, svd_driver=driver)
    rng = np.random.default_rng(perturb_seed) if perturb_seed is not None else None
    sz, tr, chi = [], [], []
    t0 = time.time()
    for k in range(n_steps + 1):
        if k:
            eng.step(1)
            if rng is not None:
                for g in eng.mps.gammas:
                    g *= 1.0 + rel * (rng.normal(size=g.shape) + 1j * rng.normal(size=g.shape))
        sz.append([eng.expectation(s, W.SZ) for s in range(n)])
        tr.append(eng.trace())
        chi.append([int(c) for c in eng.mps.bond_dims()])
        if log:
            log(k, time.time() - t0, chi[-1])
    return np.array(sz), np.array(tr), chi


def write_json(path, rec):
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(path + ".tmp", path)


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    name = args[0] if args else "xy21"
    wl = getattr(W, name)()
    n_steps = int(args[1]) if len(args) > 1 else wl["n_steps"]
    prob, _ = problem_from_workload(wl)
    n = wl["n_sites"]
    here = os.path.dirname(os.path.abspath(__file__))

    def log(k, s, chi):
        print(f"step {k} {s:.1f}s chi={chi}", flush=True)

    if "--spread" in sys.argv:
        base_sz, base_tr, _ = trajectory(prob, n, n_steps, log=log)
        rec = {"workload": name, "n_steps": n_steps, "variants": {}}
        for label, kw in (("perturb_seed1", {"perturb_seed": 1}), ("perturb_seed2", {"perturb_seed": 2}),
                          ("gesvd", {"driver": "gesvd"})):
            sz, tr, _ = trajectory(prob, n, n_steps, log=log, **kw)
            rec["variants"][label] = {"sz": np.abs(sz - base_sz).max(axis=1).tolist(),
                                      "trace": np.abs(tr - base_tr).tolist()}
            print(label, " ".join("%.1e" % e for e in rec["variants"][label]["sz"]), flush=True)
        rec["sz"] = np.max([v["sz"] for v in rec["variants"].values()], axis=0).tolist()
        rec["trace"] = np.max([v["trace"] for v in rec["variants"].values()], axis=0).tolist()
        write_json(os.path.join(here, f"{name}_spread.json"), rec)
        return

    eng = pt_tebd.Engine(prob)
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
    out = os.path.join(here, f"{name}_oracle.json")
    for k in range(1, n_steps + 1):
        eng.step(1)
        record()
        print(f"step {k} {time.time() - t0:.1f}s chi={rec['chi'][-1]}", flush=True)
        if k % 5 == 0 or k == n_steps:
            write_json(out, rec)


if __name__ == "__main__":
    main()
