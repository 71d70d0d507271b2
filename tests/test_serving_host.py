"""Host logic of the continuous-batching loop (serving.Server) on the CPU,
with the library replaced by recording fakes: admission in arrival order
under the memory budget, one batch over exactly the admitted chains, every
request stepped exactly its number of steps, read out once and freed, and a
request larger than the budget still served when nothing else runs."""
import types

import numpy as np

from paper_2201_05529_amd import serving as S
from paper_2201_05529_amd import workloads as W


class FakeLib:
    def __init__(self, sizes):
        self.sizes = sizes          # request name -> bytes
        self.live = {}              # chain id -> bytes
        self.peak = 0
        self.batches = []
        self.steps = {}
        self.reads = {}
        self.builds = []

    # binding surface used by the loop
    FP64, FP32_MIXED = 0, 1

    def build_ptmpo_batch(self, specs, dt, n_steps, k_cut, eps, xi, stream=None):
        self.builds.append([sp["n_steps"] for sp in specs])
        assert all(sp["n_steps"] <= n_steps for sp in specs)
        return [{"tensors": [("pt", sp["n_steps"])]} for sp in specs]

    def workspace_bytes(self, h_site, h_bond, rho0, dt, baths=(), chi_max=64, **kw):
        return self.sizes[len(h_site), chi_max]

    def chain_class(self):
        lib = self

        class Chain:
            count = 0

            def __init__(self, h_site, h_bond, rho0, dt, baths=(), chi_max=64, **kw):
                Chain.count += 1
                self.id = Chain.count
                self.n = len(h_site)
                self.bytes = lib.sizes[self.n, chi_max]
                lib.live[self.id] = self.bytes
                lib.peak = max(lib.peak, sum(lib.live.values()))
                lib.steps[self.id] = 0
                self.handle = self.id

            def observe(self, sites, ops):
                lib.reads[self.id] = lib.reads.get(self.id, 0) + 1
                return np.full(self.n, float(lib.steps[self.id])), 1.0

            def close(self):
                lib.live.pop(self.id, None)

        return Chain

    def batch_class(self):
        lib = self

        class Batch:
            def __init__(self, chains):
                assert sorted(c.id for c in chains) == sorted(c.id for c in chains if c.id in lib.live)
                lib.batches.append(sorted(c.id for c in chains))
                self.chains = chains
                self.open = True

            def step(self, n=1):
                assert self.open
                for c in self.chains:
                    lib.steps[c.id] += n

            def close(self):
                self.open = False

        return Batch


def _requests():
    rng = np.random.default_rng(3)
    out = []
    arrivals = [0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    for i, n in enumerate([3, 4, 3, 5, 4, 3]):
        wl = W.random_xyz_chain(rng, f"r{i}", n, n, (8, 16), int(rng.integers(2, 7)), dt=0.05, k_cut=2, xi_max=8)
        wl["arrival_s"] = arrivals[i]
        out.append(wl)
    return out


def _run(reqs, sizes, budget, monkeypatch, max_active=8):
    fake = FakeLib(sizes)
    mod = types.SimpleNamespace(build_ptmpo_batch=fake.build_ptmpo_batch, workspace_bytes=fake.workspace_bytes,
                                Chain=fake.chain_class(), Batch=fake.batch_class(), FP64=0, FP32_MIXED=1)
    monkeypatch.setattr(S, "B", mod)
    stream = types.SimpleNamespace(synchronize=lambda: None)
    res = S.Server(budget, precision=0, max_active=max_active, max_admit=3, stream=stream).run(reqs, realtime=False)
    return fake, res


def test_admission_budget_and_steps(monkeypatch):
    reqs = _requests()
    sizes = {(wl["n_sites"], wl["chi_max"]): 100 * wl["n_sites"] for wl in reqs}
    budget = 1000
    fake, res = _run(reqs, sizes, budget, monkeypatch)
    assert fake.peak <= budget
    # every request stepped exactly its steps (the fake read-out returns the
    # step count), read out once, and freed
    for wl, r in zip(reqs, res):
        assert r.done is not None and np.all(r.sz == wl["n_steps"])
        assert r.site_updates == wl["n_sites"] * wl["n_steps"]
    assert all(v == 1 for v in fake.reads.values()) and not fake.live
    # arrival order: admissions are non-decreasing in request index
    adm = [r.admitted for r in res]
    assert adm == sorted(adm)
    # PT-MPOs built in groups of at most three, each at its request's length
    assert all(len(g) <= 3 for g in fake.builds)
    assert sorted(x for g in fake.builds for x in g) == sorted(wl["n_steps"] for wl in reqs)
    # batches re-formed only over chains alive at the time
    assert all(len(b) >= 1 for b in fake.batches)


def test_oversized_request_runs_alone(monkeypatch):
    reqs = _requests()[:3]
    sizes = {(wl["n_sites"], wl["chi_max"]): 100 for wl in reqs}
    big = (reqs[1]["n_sites"], reqs[1]["chi_max"])
    sizes[big] = 5000
    fake, res = _run(reqs, sizes, 1000, monkeypatch)
    assert all(r.done is not None for r in res)
    # handles are created in admission order: request 1 is chain 2.  It
    # waited for request 0 to finish, ran alone, and request 2 waited
    # behind it (admission keeps arrival order)
    assert fake.peak == 5000
    assert all(b == [2] for b in fake.batches if 2 in b)
    assert res[0].done <= res[1].admitted <= res[1].done <= res[2].admitted
