#!/usr/bin/env python3
"""Throughput of the PT-TEBD hot path on one GPU.

One step = one full time step Delta t of the chain (Sec. II, the step of
eq. propagator-env: two chain half-steps of three Trotter sublayers of
two-site updates, and the absorption of every bath's PT-MPO tensor in
between) followed by one read-out of <sigma^z_n> on every site.  A
site-update is one site advanced by one Delta t, so a run of K steps of an
N-site chain counts N*K site-updates.

Default workload: the N = 21 XY chain with a bath on every site (chi <= 64,
xi <= 24, dt = 0.1, 100 steps).  The timed region runs the workload's steps
1..K from the initial state on a fresh handle, inputs and PT-MPOs already
resident in device memory; gate build and PT-MPO build/upload are timed
separately and excluded.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "site-updates/s, XY N=21 chi=64, FP32-mixed vs FP64 at <=1e-4 err; p50/p99 latency"


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100, help="timed steps (the workload has 100)")
    p.add_argument("--warmup", type=int, default=3, help="untimed steps on a throwaway handle")
    p.add_argument("--workload", default="xy21")
    p.add_argument("--precision", default="fp64", choices=["fp64"])
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="time budget of the oracle CPU baseline (0 disables it)")
    p.add_argument("--chains", type=int, default=1,
                   help="independent copies of the workload, each on a stream of its own (value = their total)")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="before the workload, run one element-wise copy kernel that reads and writes MIB MiB "
                        "(the reference for hardware byte counters)")
    p.add_argument("--kernel", default="eigensolver", choices=["eigensolver", "gemm", "none"],
                   help="kernel class timed per launch with HIP events during the timed region "
                        "(the dominant one) for the roofline object")
    return p.parse_args()


KERNEL_CLASS = {"none": 0, "eigensolver": 1, "gemm": 2}
# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6   # FP64 vector and FP64 dense matrix
PROFILES = os.path.join(ROOT, "profiles")


def kernel_sources(kind):
    csrc = os.path.join(ROOT, "paper_2201_05529_amd", "csrc")
    files = {"eigensolver": ["heev.h", "device_common.h"], "gemm": ["gemm.h", "bond_kernels.h", "device_common.h"]}
    return [os.path.join(csrc, f) for f in files[kind]]


def traffic_from_profiles(kind, launches_per_step):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources (else None)."""
    import hashlib
    path = os.path.join(PROFILES, f"{kind}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in kernel_sources(kind):
        with open(src, "rb") as g:
            h.update(g.read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec.get("bytes_per_launch")


def roofline(kind, ms_total, launches, flops):
    if kind == "none" or launches == 0 or ms_total <= 0.0:
        return None
    avg_s = ms_total * 1e-3 / launches
    achieved = flops / launches / avg_s * 1e-12
    bound = "alu"  # both kernels run FP64 vector arithmetic (CDNA4 has no faster FP64 matrix rate)
    return {"bound": bound, "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic_from_profiles(kind, launches),
            "kernel": {"eigensolver": "heev_solve_kernel", "gemm": "k_bond_gemm"}[kind],
            "launches": launches, "avg_launch_ms": ms_total / launches,
            "alg_flops_per_launch": flops / launches}


def library_baths(wl, n_steps):
    """PT-MPOs from the library's own builder (one per distinct parameter set)."""
    from paper_2201_05529_amd import binding as B
    cache, out = {}, []
    for b in wl["baths"]:
        key = (b["alpha"], b["wc"], b["temperature"], b["k_cut"], b["cutoff"], b["coupling_op"].tobytes())
        if key not in cache:
            cache[key] = B.build_ptmpo(b["alpha"], b["wc"], b["temperature"], wl["dt"], n_steps, b["k_cut"],
                                       wl["eps_tempo"], wl["xi_max"], b["coupling_op"], cutoff=b["cutoff"])
        out.append({"site": b["site"], "tensors": cache[key]["tensors"]})
    return out


def make_chain(wl, baths, stream=None):
    from paper_2201_05529_amd import binding as B
    return B.Chain(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths, chi_max=wl["chi_max"],
                   xi_max=wl["xi_max"], eps=wl["eps"], lindblad=wl.get("lindblad"), stream=stream)


def cpu_baseline(wl, seconds):
    """The oracle (FP64 NumPy) on the host, steps 1..S of the same workload
    until the time budget is spent (at least one step)."""
    from oracle import pt_tebd
    from oracle.build import problem_from_workload
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    n = wl["n_sites"]
    prob, _ = problem_from_workload(wl, n_steps=wl["n_steps"])
    eng = pt_tebd.Engine(prob)
    steps = 0
    t0 = time.perf_counter()
    while True:
        eng.step(1)
        for s in range(n):
            eng.expectation(s, np.array([[1, 0], [0, -1]], dtype=np.complex128))
        steps += 1
        t = time.perf_counter() - t0
        if t >= seconds or steps >= wl["n_steps"]:
            break
    chi = max(eng.mps.bond_dims())
    return {"value": n * steps / t, "unit": "site-updates/s", "cores": int(threads), "kind": "oracle",
            "sample": f"steps 1..{steps} of the {wl['n_steps']}-step workload from the initial state "
                      f"(max chi reached {chi}; later steps at chi={wl['chi_max']} cost more), "
                      f"{t:.1f} s wall"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): the PT-TEBD path here "
              f"has no multi-GPU form; see the sharding notes in the design document", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_2201_05529_amd import binding as B
    from paper_2201_05529_amd import workloads as W
    B.lib()  # fails loudly if the HIP library is missing
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    wl = getattr(W, args.workload)()
    n = wl["n_sites"]
    horizon = max(args.steps, args.warmup, wl["n_steps"])
    t0 = time.perf_counter()
    baths = library_baths(wl, horizon)
    t_ptmpo = time.perf_counter() - t0
    sites = np.arange(n, dtype=np.int32)
    ops = np.array([W.SZ] * n)

    # warm-up on a throwaway handle
    if args.warmup > 0:
        ch = make_chain(wl, baths)
        for _ in range(args.warmup):
            ch.step(1)
            ch.observe(sites, ops)
        ch.close()
        del ch

    t0 = time.perf_counter()
    n_chains = max(1, args.chains)
    # one chain on the current stream; further copies on streams of their
    # own (default priority), so their launches overlap on the device
    streams = [None] + [torch.cuda.Stream() for _ in range(n_chains - 1)]
    chains = [make_chain(wl, baths, stream=st) for st in streams]
    ch = chains[0]
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    ch.kernel_timing(KERNEL_CLASS[args.kernel])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    peak_chi, peak_xi = 0, 0
    for k in range(args.steps):
        for c in chains:
            c.step(1)
        for c in chains:
            vals, tr = c.observe(sites, ops)
        chi, xi = ch.bond_dims()
        peak_chi, peak_xi = max(peak_chi, int(chi.max())), max(peak_xi, int(xi.max()))
        if (k + 1) % 10 == 0:
            print(f"bench: step {k + 1}/{args.steps} {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_k, launches_k, flops_k = ch.kernel_timing_read()
    value = n_chains * n * args.steps / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={n} XY chain, a bath on every site, chi<={wl['chi_max']}, "
                               f"xi<={wl['xi_max']}, dt={wl['dt']}, steps 1..{args.steps}, FP64 plain"
                               + (f", {n_chains} independent copies on {n_chains} streams" if n_chains > 1 else ""),
                   "precision": args.precision, "peak_chi": peak_chi, "peak_xi": peak_xi,
                   "trace": [tr.real, tr.imag], "ptmpo_build_s": t_ptmpo, "create_s": t_create},
    }
    rl = roofline(args.kernel, ms_k, launches_k, flops_k)
    if rl is not None:
        out["roofline"] = rl
    for c in chains:
        c.close()
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
