"""Shared test helpers: build the same problem for the oracle and the library."""
import os

import numpy as np

from oracle.build import problem_from_workload
from oracle import pt_tebd as opt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_library():
    from paper_2201_05529_amd import build_lib
    if not os.path.exists(build_lib.LIB):
        build_lib.build()
    return build_lib.LIB


def oracle_problem(wl, n_steps=None, form="tempo"):
    prob, cache = problem_from_workload(wl, form=form, n_steps=n_steps)
    return prob


def library_chain(wl, prob, precision=0, **kw):
    """Library handle fed with the oracle's PT-MPO tensors and caps."""
    from paper_2201_05529_amd import binding as B
    baths = [{"site": b["site"], "tensors": b["tensors"], "caps": b["caps"], "initial": b.get("initial")}
             for b in prob.baths]
    xi = max([max(p.shape[1] for p in b["tensors"]) for b in prob.baths] + [1])
    return B.Chain(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths,
                   chi_max=wl["chi_max"], xi_max=max(xi, 1), eps=wl["eps"], precision=precision,
                   lindblad=wl.get("lindblad"), **kw)


def run_both(wl, n_steps, ops, precision=0, form="tempo", oracle_mode="ch"):
    """Step both paths n_steps, observing `ops` (list of (site, op)) at every
    step; returns (gpu [steps+1, n_ops], oracle [steps+1, n_ops], gpu trace,
    oracle trace, chain)."""
    prob = oracle_problem(wl, n_steps=n_steps, form=form)
    eng = opt.Engine(prob, mode=oracle_mode)
    ch = library_chain(wl, prob, precision=precision)
    sites = [s for s, _ in ops]
    mats = np.array([o for _, o in ops])
    g, o, gt, ot = [], [], [], []
    for k in range(n_steps + 1):
        if k > 0:
            ch.step(1)
            eng.step(1)
        v, tr = ch.observe(sites, mats)
        g.append(v)
        gt.append(tr)
        o.append([eng.expectation(s, op) for s, op in ops])
        ot.append(eng.trace())
    return np.array(g), np.array(o), np.array(gt), np.array(ot), ch, eng


def oracle_sensitivity(prob, n_steps, ops, seeds=(1, 2), rel=1e-15):
    """Per-step spread of the oracle's own observables under rounding-level
    perturbations: after every step every entry of every site tensor is
    multiplied by (1 + rel * complex normal), as a different floating-point
    implementation of the same steps perturbs them.  Returns (base
    [steps+1, n_ops], envelope [steps+1]) with envelope[k] = max over seeds
    and ops of the deviation from the unperturbed run.  No other
    floating-point implementation can be expected to reproduce the oracle
    more closely than this."""
    def run(seed):
        eng = opt.Engine(prob)
        rng = np.random.default_rng(seed)
        out = []
        for k in range(n_steps + 1):
            if k:
                eng.step(1)
                if seed:
                    for g in eng.mps.gammas:
                        g *= 1.0 + rel * (rng.normal(size=g.shape) + 1j * rng.normal(size=g.shape))
            out.append([eng.expectation(s, op) for s, op in ops])
        return np.array(out)
    base = run(0)
    env = np.zeros(n_steps + 1)
    for seed in seeds:
        env = np.maximum(env, np.abs(run(seed) - base).max(axis=1))
    return base, env
