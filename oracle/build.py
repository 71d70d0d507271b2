"""Turn a workload description (plain dict of arrays and bath parameters)
into oracle inputs: eta by quadrature (bath.py) and the PT-MPO by the
oracle's own builders (ptmpo.py).  Baths with identical parameters share
one PT-MPO, as the paper does for the 21-site chain (Sec. IV).
"""
import numpy as np

from . import bath as bathmod
from . import ptmpo
from .pt_tebd import Problem


def bath_key(b):
    return (b["alpha"], b["wc"], b["temperature"], b["k_cut"], b.get("cutoff", "exp"),
            tuple(np.asarray(b["coupling_op"]).reshape(-1).tolist()))


def build_ptmpo(b, dt, n_steps, eps, xi_max, form="tempo"):
    """Returns dict(tensors, caps, diagonal, eta)."""
    eta = bathmod.eta_coefficients(b["alpha"], b["wc"], b["temperature"], dt, b["k_cut"],
                                   b.get("cutoff", "exp"))
    sigma, diagonal = ptmpo.coupling_eigensystem(b["coupling_op"])
    if form == "history":
        tensors = ptmpo.history_mpo(eta, sigma, n_steps)
    else:
        tensors = ptmpo.tempo_mpo(eta, sigma, n_steps, eps, xi_max)
    if not diagonal:
        tensors = ptmpo.to_computational_basis(tensors, b["coupling_op"])
    d = int(round(np.sqrt(len(sigma) ** 2)))
    return {"tensors": tensors, "caps": ptmpo.caps(tensors, d), "diagonal": diagonal, "eta": eta}


def problem_from_workload(wl, form="tempo", n_steps=None, pt_cache=None):
    n_steps = wl["n_steps"] if n_steps is None else n_steps
    cache = {} if pt_cache is None else pt_cache
    baths = []
    for b in wl["baths"]:
        key = bath_key(b) + (wl["dt"], n_steps, wl["eps_tempo"], wl["xi_max"], form)
        if key not in cache:
            cache[key] = build_ptmpo(b, wl["dt"], n_steps, wl["eps_tempo"], wl["xi_max"], form)
        pt = cache[key]
        baths.append({"site": b["site"], "tensors": pt["tensors"], "caps": pt["caps"]})
    lindblad = wl.get("lindblad")
    prob = Problem(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths,
                   lindblad=lindblad, chi_max=wl["chi_max"], eps=wl["eps"], d=wl["d"])
    return prob, cache
