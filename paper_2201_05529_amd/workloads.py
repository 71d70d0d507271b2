"""Seeded synthetic workloads: spin-chain problem definitions.

This module only writes down problem inputs -- chain Hamiltonians as
matrices (Sec. III eq. xyz-spin-chain, Sec. IV eq. xy-spin-chain), initial
product states, bath parameters, numerical caps -- and draws the random
parameters of the batched and serving workloads from a seeded generator.
It holds none of the method's arithmetic, imports nothing from the library
or the test oracle, and is the one module both sides read.

Workloads (scaled analogues of the paper's experiments, Sec. III and IV):
  xyz3      N=3 XYZ (J = 1.3, 0.7, 1.2), bath on the first site via sigma^z
  xyz5      N=5 XYZ, hot (T=2.0) bath on the first site, cold (T=0.5) on the last
  xy21      N=21 isotropic XY chain with unit field, a bath on every site,
            centre spin up (the headline workload)
  batch256  256 independent XYZ chains with randomised sizes and parameters
  serving   Poisson request stream of randomised chains
"""
import numpy as np

MASTER_SEED = 220105529

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
UP = np.array([[1, 0], [0, 0]], dtype=np.complex128)
DOWN = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def xyz_bond(jx, jy, jz):
    """J^x s^x s^x + J^y s^y s^y + J^z s^z s^z with s = sigma/2 (natural
    two-site order)."""
    return 0.25 * (jx * np.kron(SX, SX) + jy * np.kron(SY, SY) + jz * np.kron(SZ, SZ))


def bath(site, alpha, wc, temperature, k_cut, coupling=SZ, cutoff="exp"):
    return {"site": int(site), "alpha": float(alpha), "wc": float(wc),
            "temperature": float(temperature), "k_cut": int(k_cut),
            "coupling_op": np.asarray(coupling, dtype=np.complex128), "cutoff": cutoff}


def make_chain(name, n_sites, bond_terms, field, rho0, dt, n_steps, baths,
               chi_max, xi_max, eps=1e-7, eps_tempo=1e-7):
    h_site = np.array([0.5 * field[n] * SZ for n in range(n_sites)], dtype=np.complex128)
    h_bond = np.array(bond_terms, dtype=np.complex128).reshape(n_sites - 1, 4, 4) \
        if n_sites > 1 else np.zeros((0, 4, 4), dtype=np.complex128)
    return {"name": name, "n_sites": n_sites, "d": 2, "dt": float(dt), "n_steps": int(n_steps),
            "h_site": h_site, "h_bond": h_bond, "lindblad": None,
            "rho0": np.array(rho0, dtype=np.complex128), "baths": list(baths),
            "chi_max": int(chi_max), "xi_max": int(xi_max), "eps": float(eps),
            "eps_tempo": float(eps_tempo)}


def xyz3():
    n = 3
    bonds = [xyz_bond(1.3, 0.7, 1.2)] * (n - 1)
    rho0 = [UP, DOWN, DOWN]
    return make_chain("xyz3", n, bonds, [0.0] * n, rho0, dt=0.1, n_steps=40,
                      baths=[bath(0, 0.08, 4.0, 1.6, 10)], chi_max=16, xi_max=16)


def xyz5():
    n = 5
    bonds = [xyz_bond(1.3, 0.7, 1.2)] * (n - 1)
    rho0 = [UP] + [DOWN] * (n - 1)
    return make_chain("xyz5", n, bonds, [0.0] * n, rho0, dt=0.05, n_steps=200,
                      baths=[bath(0, 0.16, 4.0, 2.0, 20), bath(n - 1, 0.16, 4.0, 0.5, 20)],
                      chi_max=64, xi_max=40)


def xy21():
    n = 21
    bonds = [xyz_bond(1.0, 1.0, 0.0)] * (n - 1)
    rho0 = [DOWN] * n
    rho0[n // 2] = UP
    return make_chain("xy21", n, bonds, [1.0] * n, rho0, dt=0.1, n_steps=100,
                      baths=[bath(s, 0.05, 4.0, 1.0, 10) for s in range(n)],
                      chi_max=64, xi_max=24)


def random_xyz_chain(rng, name, n_lo, n_hi, chi_caps, n_steps, dt=0.05, k_cut=20, xi_max=24):
    n = int(rng.integers(n_lo, n_hi + 1))
    jx, jy, jz = rng.uniform(0.5, 1.5, size=3)
    alpha = rng.uniform(0.02, 0.2)
    temperature = rng.uniform(0.5, 3.0)
    chi_max = int(rng.choice(chi_caps))
    bonds = [xyz_bond(jx, jy, jz)] * (n - 1)
    rho0 = [UP] + [DOWN] * (n - 1)
    return make_chain(name, n, bonds, [0.0] * n, rho0, dt=dt, n_steps=n_steps,
                      baths=[bath(s, alpha, 4.0, temperature, k_cut) for s in range(n)],
                      chi_max=chi_max, xi_max=xi_max)


def batch256(n_chains=256, n_steps=100):
    rng = np.random.default_rng(MASTER_SEED)
    return [random_xyz_chain(rng, f"batch{i}", 4, 16, (16, 32, 64), n_steps)
            for i in range(n_chains)]


def serving_stream(duration_s=60.0, rate_hz=50.0):
    """Poisson arrivals; each request is a random XYZ chain."""
    rng_t = np.random.default_rng(MASTER_SEED + 1)
    rng_r = np.random.default_rng(MASTER_SEED + 2)
    t, out = 0.0, []
    while True:
        t += rng_t.exponential(1.0 / rate_hz)
        if t > duration_s:
            break
        steps = int(rng_r.integers(50, 401))
        req = random_xyz_chain(rng_r, f"req{len(out)}", 3, 32, (16, 32, 64, 128), steps,
                               xi_max=32)
        req["arrival_s"] = t
        out.append(req)
    return out


def random_small_chain(seed, n_sites, n_steps=4, with_bath_sites=(0,), k_cut=3,
                       chi_max=None, xi_max=None, eps=1e-12, dt=0.1, field=True,
                       random_state=True):
    """Small random problems for parity and property tests: random XYZ
    couplings and fields, random mixed single-site states."""
    rng = np.random.default_rng(MASTER_SEED + 1000 + seed)
    j = rng.uniform(0.3, 1.5, size=(max(n_sites - 1, 0), 3))
    bonds = [xyz_bond(*j[b]) for b in range(n_sites - 1)]
    fields = rng.uniform(-1.0, 1.0, size=n_sites) if field else np.zeros(n_sites)
    rho0 = []
    for _ in range(n_sites):
        if random_state:
            m = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
            r = m @ m.conj().T
            rho0.append(r / np.trace(r))
        else:
            rho0.append(UP)
    baths = [bath(s, rng.uniform(0.05, 0.3), 4.0, rng.uniform(0.5, 2.0), k_cut)
             for s in with_bath_sites]
    return make_chain(f"small{seed}", n_sites, bonds, fields, rho0, dt=dt, n_steps=n_steps,
                      baths=baths, chi_max=chi_max if chi_max else 256,
                      xi_max=xi_max if xi_max else 4 ** max(k_cut, 1), eps=eps, eps_tempo=eps)
