#!/usr/bin/env python3
"""Throughput of the PT-TEBD hot path on one GPU.

One step = one full time step Delta t of the chain (Sec. II, the step of
eq. propagator-env: two chain half-steps of three Trotter sublayers of
two-site updates, and the absorption of every bath's PT-MPO tensor in
between) followed by one read-out of <sigma^z_n> on every site.  A
site-update is one site advanced by one Delta t, so K steps of an N-site
chain count N*K site-updates.

Default workload: the N = 21 XY chain with a bath on every site (chi <= 64,
xi <= 24, dt = 0.1, 100 steps), run twice on fresh handles over the same
window, steps 1..K from the initial state (K = 100, the whole workload, by
default): once in the FP32-mixed form (complex contractions in single
precision on the matrix cores, eigensolvers, singular values, gates, PT
absorption and the log-scale in double precision) and once in plain FP64.
The headline value is the FP32-mixed rate; the FP64 rate, the speed-up,
each form's largest deviation from the stored oracle trajectory and the
per-step latency quantiles sit beside it.  Inputs and PT-MPOs are resident
in device memory when the timed region starts; the PT-MPO build (on the
GPU) and handle creation are timed separately and excluded.

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
# MI355X published dense peaks
PEAK_TFLOPS = {"fp64": 78.6, "fp32_mixed": 157.3}
PROFILES = os.path.join(ROOT, "profiles")
GOLDEN = os.path.join(ROOT, "tests", "golden")
KERNEL_CLASS = {"none": 0, "eigensolver": 1, "gemm": 2}


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100, help="timed steps from the initial state (the workload has 100)")
    p.add_argument("--warmup", type=int, default=2, help="untimed steps on a throwaway handle per form")
    p.add_argument("--workload", default="xy21", help="xy21, xyz5, xyz3, batched (many independent chains) or serving (the request stream)")
    p.add_argument("--precision", default="both", choices=["both", "fp64", "fp32_mixed"],
                   help="forms to run; with both, value is the FP32-mixed rate")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="time budget of each oracle CPU baseline run (1 thread, all cores; 0 disables them)")
    p.add_argument("--chains", type=int, default=256,
                   help="with --workload batched: number of independent chains in the batch")
    p.add_argument("--requests", type=int, default=24, help="with --workload serving: requests taken from the stream")
    p.add_argument("--steps-scale", type=float, default=0.1,
                   help="with --workload serving: factor on each request's step count")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="before the workload, run one element-wise copy kernel that reads and writes MIB MiB "
                        "(the reference for hardware byte counters)")
    p.add_argument("--kernel", default="eigensolver", choices=["eigensolver", "gemm", "none"],
                   help="kernel class timed per launch with HIP events during the headline form's timed region "
                        "(the dominant one) for the roofline object")
    return p.parse_args()


def kernel_sources(kind):
    csrc = os.path.join(ROOT, "paper_2201_05529_amd", "csrc")
    files = {"eigensolver": ["heev.h", "device_common.h"], "gemm": ["gemm.h", "gemm_mfma.h", "bond_kernels.h",
                                                                  "device_common.h"]}
    return [os.path.join(csrc, f) for f in files[kind]]


def traffic_from_profiles(kind):
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


def kernel_roofline(kind, ms_total, launches, flops):
    """The dominant kernel alone: algorithmic flops per launch / average
    launch duration (HIP events on the handle's stream)."""
    if kind == "none" or launches == 0 or ms_total <= 0.0:
        return None
    avg_s = ms_total * 1e-3 / launches
    achieved = flops / launches / avg_s * 1e-12
    peak = PEAK_TFLOPS["fp64"]  # the eigensolver runs FP64 vector arithmetic in both forms
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic_from_profiles(kind),
            # the eigensolver's timed region: its tridiagonal reduction and
            # stages 2-4, two kernels launched back to back on the stream
            "kernel": {"eigensolver": "heev_tridiag_kernel+heev_solve_kernel", "gemm": "k_bond_gemm"}[kind],
            "launches": launches, "avg_launch_ms": ms_total / launches, "alg_flops_per_launch": flops / launches}


def composite_roofline(model_flops, elapsed_s, precision):
    """The whole step: T_ideal = (F_a1 + F_a2 + F_a3 + F_a4) / matrix-core peak
    of the form's contraction type, against the measured time."""
    f = float(np.sum(model_flops))
    peak = PEAK_TFLOPS[precision] * 1e12
    t_ideal = f / peak
    return {"model_flops": f, "F_a1_a4": [float(x) for x in model_flops], "peak_tflops": PEAK_TFLOPS[precision],
            "achieved_tflops": f / elapsed_s * 1e-12, "t_ideal_s": t_ideal, "t_measured_s": elapsed_s,
            "frac": t_ideal / elapsed_s}


def library_baths(wl, n_steps):
    """PT-MPOs from the library's GPU builder, one per distinct parameter set."""
    from paper_2201_05529_amd import binding as B
    keys, params = [], []
    for b in wl["baths"]:
        key = (b["alpha"], b["wc"], b["temperature"], b["k_cut"], b["cutoff"], b["coupling_op"].tobytes())
        if key not in keys:
            keys.append(key)
            params.append(b)
    built = {}
    by_k = {}
    for key, b in zip(keys, params):
        by_k.setdefault(b["k_cut"], []).append((key, b))
    for k_cut, items in by_k.items():
        pts = B.build_ptmpo_batch([{"alpha": b["alpha"], "wc": b["wc"], "temperature": b["temperature"],
                                    "coupling_op": b["coupling_op"], "cutoff": b["cutoff"]} for _, b in items],
                                  wl["dt"], n_steps, k_cut, wl["eps_tempo"], wl["xi_max"])
        for (key, _), pt in zip(items, pts):
            built[key] = pt
    out = []
    for b in wl["baths"]:
        key = (b["alpha"], b["wc"], b["temperature"], b["k_cut"], b["cutoff"], b["coupling_op"].tobytes())
        out.append({"site": b["site"], "tensors": built[key]["tensors"]})
    return out


def make_chain(wl, baths, precision):
    from paper_2201_05529_amd import binding as B
    prec = B.FP32_MIXED if precision == "fp32_mixed" else B.FP64
    return B.Chain(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths, chi_max=wl["chi_max"],
                   xi_max=wl["xi_max"], eps=wl["eps"], lindblad=wl.get("lindblad"), precision=prec)


def load_golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    sz = np.array(g["sz_re"]) + 1j * np.array(g["sz_im"])
    tr = np.array(g["trace_re"]) + 1j * np.array(g["trace_im"])
    spread = None
    sp = os.path.join(GOLDEN, f"{name}_spread.json")
    if os.path.exists(sp):
        with open(sp) as f:
            spread = np.array(json.load(f)["sz"])
    return sz, tr, spread


def run_form(wl, baths, precision, args, timed_kernel):
    import torch
    n = wl["n_sites"]
    sites = np.arange(n, dtype=np.int32)
    from paper_2201_05529_amd import workloads as W
    ops = np.array([W.SZ] * n)
    if args.warmup > 0:
        ch = make_chain(wl, baths, precision)
        for _ in range(args.warmup):
            ch.step(1)
            ch.observe(sites, ops)
        ch.close()
    t0 = time.perf_counter()
    ch = make_chain(wl, baths, precision)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    ch.kernel_timing(KERNEL_CLASS[timed_kernel])
    ch.model_flops(reset=True)
    torch.cuda.synchronize()
    sz, tr, lat = [], [], []
    peak_chi = peak_xi = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        ch.step(1)
        vals, trace = ch.observe(sites, ops)   # copies to the host: the step has finished
        lat.append(time.perf_counter() - ts)
        sz.append(vals)
        tr.append(trace)
        if (k + 1) % 20 == 0:
            print(f"bench[{precision}]: step {k + 1}/{args.steps} {time.perf_counter() - t0:.2f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    chi, xi = ch.bond_dims()
    peak_chi, peak_xi = int(chi.max()), int(xi.max())
    ms_k, launches_k, flops_k = ch.kernel_timing_read()
    mf = ch.model_flops()
    ch.close()
    lat = np.array(lat) * 1e3
    return {"value": n * args.steps / elapsed, "elapsed_s": elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
            "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                "max": float(lat.max())},
            "create_s": t_create, "peak_chi": peak_chi, "peak_xi": peak_xi,
            "sz": np.array(sz), "trace": np.array(tr), "kernel": (ms_k, launches_k, flops_k), "model_flops": mf}


def errors_vs_golden(res, golden, steps):
    if golden is None:
        return None
    gsz, gtr, spread = golden
    k = min(steps, gsz.shape[0] - 1)
    e_sz = np.abs(res["sz"][:k] - gsz[1:k + 1]).max(axis=1)
    e_tr = np.abs(res["trace"][:k] - gtr[1:k + 1])
    out = {"steps_compared": k, "max_dsz": float(e_sz.max()), "max_dtrace": float(e_tr.max()),
           "max_dsz_steps_1_20": float(e_sz[:20].max()), "max_dtrace_steps_1_20": float(e_tr[:20].max())}
    if spread is not None:
        m = min(k, len(spread) - 1)
        out["oracle_spread_sz_steps_1_%d" % m] = float(np.max(spread[1:m + 1]))
    return out


def cpu_baseline(wl, seconds):
    """The oracle (FP64 NumPy) on the host, steps 1..S of the same workload
    from the initial state until the time budget is spent (at least one
    step), once with one BLAS thread and once with every host core."""
    from oracle import pt_tebd
    from oracle.build import problem_from_workload
    from threadpoolctl import threadpool_info, threadpool_limits
    n = wl["n_sites"]
    prob, _ = problem_from_workload(wl, n_steps=wl["n_steps"])
    sz_op = np.array([[1, 0], [0, -1]], dtype=np.complex128)

    def run():
        eng = pt_tebd.Engine(prob)
        steps = 0
        t0 = time.perf_counter()
        while True:
            eng.step(1)
            for s in range(n):
                eng.expectation(s, sz_op)
            steps += 1
            t = time.perf_counter() - t0
            if t >= seconds or steps >= wl["n_steps"]:
                return steps, t, max(eng.mps.bond_dims())

    all_threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        s1, t1, chi1 = run()
    sa, ta, chia = run()
    return {"value": n * sa / ta, "unit": "site-updates/s", "cores": int(all_threads), "kind": "oracle",
            "sample": f"steps 1..{sa} of the {wl['n_steps']}-step workload from the initial state (max chi reached "
                      f"{chia}; the GPU window runs further, to chi={wl['chi_max']}, where a step costs more), "
                      f"{ta:.1f} s wall, NumPy/LAPACK with {all_threads} BLAS threads",
            "value_1_thread": n * s1 / t1,
            "sample_1_thread": f"steps 1..{s1}, {t1:.1f} s wall, one BLAS thread"}


def run_batched(args):
    """Many independent chains (the batched workload: chains of 4..16 sites
    with their own couplings, baths and bond caps) advanced together through
    one batch: one launch per kernel of a sublayer over every chain's bonds,
    one time step captured in a HIP graph on the first step (untimed) and
    replayed for the timed steps."""
    import torch
    from paper_2201_05529_amd import binding as B
    from paper_2201_05529_amd import workloads as W
    n_chains = args.chains
    wls = W.batch256(n_chains=n_chains, n_steps=args.steps + 1)
    horizon = args.steps + 1
    prec = B.FP32_MIXED if args.precision in ("both", "fp32_mixed") else B.FP64
    t0 = time.perf_counter()
    specs = [{"alpha": wl["baths"][0]["alpha"], "wc": wl["baths"][0]["wc"], "temperature": wl["baths"][0]["temperature"],
              "coupling_op": wl["baths"][0]["coupling_op"], "cutoff": wl["baths"][0]["cutoff"]} for wl in wls]
    pts = B.build_ptmpo_batch(specs, wls[0]["dt"], horizon, wls[0]["baths"][0]["k_cut"], wls[0]["eps_tempo"],
                              wls[0]["xi_max"])
    torch.cuda.synchronize()
    t_ptmpo = time.perf_counter() - t0
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    chains = []
    for wl, pt in zip(wls, pts):
        baths = [{"site": b["site"], "tensors": pt["tensors"]} for b in wl["baths"]]
        chains.append(B.Chain(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths, chi_max=wl["chi_max"],
                              xi_max=wl["xi_max"], eps=wl["eps"], precision=prec, stream=stream))
    batch = B.Batch(chains)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        batch.step(1)   # captures the graph
    stream.synchronize()
    t_first = time.perf_counter() - t0
    for c in chains:
        c.model_flops(reset=True)
    site_updates = sum(wl["n_sites"] for wl in wls) * args.steps
    lat = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        batch.step(1)
        stream.synchronize()
        lat.append(time.perf_counter() - ts)
        if (k + 1) % 10 == 0:
            print(f"bench[batched]: step {k + 1}/{args.steps} {time.perf_counter() - t0:.2f} s", file=sys.stderr,
                  flush=True)
    elapsed = time.perf_counter() - t0
    mf = np.sum([c.model_flops() for c in chains], axis=0)
    traces = []
    for c, wl in zip(chains, wls):
        _, tr = c.observe(np.arange(wl["n_sites"], dtype=np.int32), np.array([W.SZ] * wl["n_sites"]))
        traces.append(tr)
    batch.close()
    for c in chains:
        c.close()
    lat = np.array(lat) * 1e3
    form = "fp32_mixed" if prec == B.FP32_MIXED else "fp64"
    caps = [wl["chi_max"] for wl in wls]
    out = {
        "metric": "site-updates/s, batched independent chains (all chains together)",
        "value": site_updates / elapsed, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64-mfma+f64" if form == "fp32_mixed" else "c128", "data": "synthetic",
        "config": {"workload": f"batch{n_chains}: {n_chains} XYZ chains, N~U{{4..16}} ({sum(w['n_sites'] for w in wls)} "
                               f"sites), chi cap in {{16,32,64}} ({caps.count(16)}/{caps.count(32)}/{caps.count(64)}), "
                               f"xi<=24, K=20, dt=0.05, a bath on every site; timed steps 2..{args.steps + 1} "
                               f"(step 1 captures the HIP graph, {t_first:.2f} s)",
                   "form": form, "ptmpo_build_s": t_ptmpo, "ptmpo_builds": n_chains, "create_s": t_create,
                   "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                   "trace_range": [float(np.min(np.real(traces))), float(np.max(np.real(traces)))],
                   "composite_roofline": composite_roofline(mf, elapsed, form)},
    }
    print(json.dumps(out), flush=True)


def run_serving(args):
    """The request stream of the serving workload (Poisson arrivals at
    50 requests/s; N ~ U{3..32}, chi cap in {16, 32, 64, 128}, xi <= 32,
    dt = 0.05, K = 20, a bath on every site) through the continuous-batching
    loop: the first --requests requests, each request's step count scaled by
    --steps-scale (the full stream offers far more work than one GPU
    sustains: about 3,900 site-updates per request at 50 requests/s)."""
    import torch
    from paper_2201_05529_amd import binding as B
    from paper_2201_05529_amd import serving as S
    from paper_2201_05529_amd import workloads as W
    reqs = W.serving_stream()[: args.requests]
    full_steps = [wl["n_steps"] for wl in reqs]
    for wl in reqs:
        wl["n_steps"] = max(1, int(round(wl["n_steps"] * args.steps_scale)))
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    prec = B.FP32_MIXED if args.precision in ("both", "fp32_mixed") else B.FP64
    srv = S.Server(budget, precision=prec, max_active=256, max_admit=64)

    def log(msg):
        print("bench[serving]: " + msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=True, log=log)
    wall = time.perf_counter() - t0
    lat = np.array([r.latency for r in res])
    wait = np.array([r.admitted - r.arrival for r in res])
    su = sum(r.site_updates for r in res)
    offered = sum(wl["n_sites"] * wl["n_steps"] for wl in reqs) / max(reqs[-1]["arrival_s"], 1e-9)
    caps = [wl["chi_max"] for wl in reqs]
    form = "fp32_mixed" if prec == B.FP32_MIXED else "fp64"
    out = {
        "metric": "serving: p50/p99 request latency and site-updates/s under continuous batching",
        "value": su / wall, "unit": "site-updates/s", "n_gpus": 1, "steps": int(sum(wl["n_steps"] for wl in reqs)),
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64-mfma+f64" if form == "fp32_mixed" else "c128", "data": "synthetic",
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "config": {"workload": f"serving: first {len(reqs)} requests of the Poisson stream (50/s), N~U{{3..32}}, "
                               f"chi cap in {{16,32,64,128}} ({caps.count(16)}/{caps.count(32)}/{caps.count(64)}/"
                               f"{caps.count(128)}), xi<=32, K=20, dt=0.05, steps U{{50..400}} scaled by "
                               f"{args.steps_scale} (mean {np.mean([wl['n_steps'] for wl in reqs]):.1f}, "
                               f"unscaled mean {np.mean(full_steps):.1f})",
                   "form": form, "budget_bytes": budget, "wall_s": wall, "site_updates": su,
                   "offered_site_updates_per_s": offered,
                   "latency_s": {"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                                 "p99": float(np.percentile(lat, 99)), "max": float(lat.max())},
                   "queue_wait_s": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
                   "latency_definition": "completion (final observables on the host) minus arrival; includes "
                                         "queueing, the PT-MPO build and every step"},
    }
    print(json.dumps(out), flush=True)


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
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "serving":
        run_serving(args)
        return
    wl = getattr(W, args.workload)()
    n = wl["n_sites"]
    horizon = max(args.steps, args.warmup, wl["n_steps"])
    t0 = time.perf_counter()
    baths = library_baths(wl, horizon)
    torch.cuda.synchronize()
    t_ptmpo = time.perf_counter() - t0
    forms = ["fp32_mixed", "fp64"] if args.precision == "both" else [args.precision]
    head = forms[0]
    golden = load_golden(args.workload)
    res = {}
    for f in forms:
        res[f] = run_form(wl, baths, f, args, args.kernel if f == head else "none")
    r = res[head]
    window = f"steps 1..{args.steps} from the initial state"
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64-mfma+f64" if head == "fp32_mixed" else "c128",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={n} chain, {len(wl['baths'])} ohmic bath(s), chi<={wl['chi_max']}, "
                               f"xi<={wl['xi_max']}, dt={wl['dt']}, {window}; value = {head} form",
                   "forms": forms, "ptmpo_build_s": t_ptmpo, "ptmpo_builder": "GPU (pt_mpo_build_ohmic_batch)"},
    }
    for f in forms:
        rf = res[f]
        out["config"][f] = {
            "site_updates_per_s": rf["value"], "ms_per_step": rf["ms_per_step"],
            "step_latency_ms": rf["step_latency_ms"], "create_s": rf["create_s"],
            "peak_chi": rf["peak_chi"], "peak_xi": rf["peak_xi"],
            "trace_final": [float(rf["trace"][-1].real), float(rf["trace"][-1].imag)],
            "error_vs_oracle": errors_vs_golden(rf, golden, args.steps),
            "composite_roofline": composite_roofline(rf["model_flops"], rf["elapsed_s"], f),
        }
    if len(forms) == 2:
        out["config"]["speedup_fp32_mixed_vs_fp64"] = res["fp32_mixed"]["value"] / res["fp64"]["value"]
        out["config"]["max_dsz_fp32_mixed_vs_fp64"] = float(np.abs(res["fp32_mixed"]["sz"] - res["fp64"]["sz"]).max())
    out["p50_ms"] = r["step_latency_ms"]["p50"]
    out["p99_ms"] = r["step_latency_ms"]["p99"]
    rl = kernel_roofline(args.kernel, *r["kernel"])
    if rl is not None:
        out["roofline"] = rl
        out["roofline"]["composite_frac"] = out["config"][head]["composite_roofline"]["frac"]
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
