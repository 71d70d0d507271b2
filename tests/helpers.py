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
    baths = [{"site": b["site"], "tensors": b["tensors"], "caps": b["caps"]} for b in prob.baths]
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
