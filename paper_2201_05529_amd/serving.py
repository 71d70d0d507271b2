"""Continuous-batching request loop over the PT-TEBD library.

Each request is one chain simulation (couplings, initial state, baths, bond
caps, number of steps).  Requests that arrive while others are being
stepped are admitted as device memory frees up: the loop keeps a device
memory budget, admits waiting requests in arrival order while their handles
fit, and advances every admitted chain together through one batch (one
launch per kernel of a sublayer over the bonds of all chains; the bond
updates of different chains are independent, as those of one sublayer are,
Sec. II.B and Appendix A.2).  After every step the finished requests are
read out (<sigma^z_n> on every site and Tr rho), their handles are freed,
and the next waiting requests are admitted; the batch is re-formed whenever
its membership changes.  A request's state stays in device memory from
admission to completion.

The PT-MPO of every bath is built on the GPU (Appendix B.1) for the
requests admitted in one round together, each at its own length, so a
request's PT-MPO and therefore its result do not depend on which requests
share its round or its batch.

All arithmetic runs in the library; this module only schedules.
"""
import collections
import time

import numpy as np

from . import binding as B

SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


class Result:
    __slots__ = ("rid", "arrival", "admitted", "done", "sz", "trace", "site_updates", "ptmpo_s", "bytes")

    def __init__(self, rid, arrival):
        self.rid, self.arrival = rid, arrival
        self.admitted = self.done = None
        self.sz = self.trace = None
        self.site_updates = 0
        self.ptmpo_s = 0.0
        self.bytes = 0

    @property
    def latency(self):
        return self.done - self.arrival


def _bath_spec(b, n_steps):
    return {"alpha": b["alpha"], "wc": b["wc"], "temperature": b["temperature"], "coupling_op": b["coupling_op"],
            "cutoff": b["cutoff"], "n_steps": n_steps}


def _distinct_baths(wl):
    """The request's distinct bath parameter sets and, per bath, its index."""
    keys, idx = [], []
    for b in wl["baths"]:
        key = (b["alpha"], b["wc"], b["temperature"], b["k_cut"], b["cutoff"], b["coupling_op"].tobytes())
        if key not in keys:
            keys.append(key)
        idx.append(keys.index(key))
    return keys, idx


class Server:
    """budget_bytes: device memory the handles of admitted requests may use
    together.  max_active: most requests in the batch at once.  max_admit:
    most requests whose PT-MPOs are built in one admission round."""

    def __init__(self, budget_bytes, precision=B.FP32_MIXED, max_active=256, max_admit=64, stream=None):
        self.budget = int(budget_bytes)
        self.precision = precision
        self.max_active = max_active
        self.max_admit = max_admit
        if stream is None:
            import torch
            # the default stream: batches re-formed every few steps issue
            # their launches directly instead of capturing a graph each time
            stream = torch.cuda.default_stream()
        self.stream = stream

    def _sync(self):
        self.stream.synchronize()

    def _build(self, group):
        """PT-MPOs of a group of requests in one GPU call per (dt, memory
        cutoff, eps, xi cap) class; each bath at its request's length."""
        out = {}
        classes = collections.OrderedDict()
        for rid, wl in group:
            keys, _ = _distinct_baths(wl)
            for key in keys:
                b = next(x for x in wl["baths"] if (x["alpha"], x["wc"], x["temperature"], x["k_cut"], x["cutoff"],
                                                     x["coupling_op"].tobytes()) == key)
                cls = (wl["dt"], b["k_cut"], wl["eps_tempo"], wl["xi_max"])
                classes.setdefault(cls, []).append((rid, key, _bath_spec(b, wl["n_steps"])))
        for (dt, k_cut, eps_t, xi), items in classes.items():
            horizon = max(spec["n_steps"] for _, _, spec in items)
            pts = B.build_ptmpo_batch([spec for _, _, spec in items], dt, horizon, k_cut, eps_t, xi,
                                      stream=self.stream)
            for (rid, key, _), pt in zip(items, pts):
                out.setdefault(rid, {})[key] = pt["tensors"]
        return out

    def _baths(self, wl, tensors):
        keys, idx = _distinct_baths(wl)
        return [{"site": b["site"], "tensors": tensors[keys[i]]} for b, i in zip(wl["baths"], idx)]

    def run(self, requests, realtime=True, log=None):
        """requests: list of workload dicts with "arrival_s" and "n_steps".
        Replays the arrivals against the wall clock (realtime) or takes them
        all at time zero.  Returns the list of Result, in request order."""
        order = sorted(range(len(requests)), key=lambda i: requests[i].get("arrival_s", 0.0) if realtime else 0.0)
        pending = collections.deque(order)
        waiting = collections.deque()
        results = [Result(i, requests[i].get("arrival_s", 0.0) if realtime else 0.0) for i in range(len(requests))]
        built = {}                 # rid -> {bath key: tensors}
        active = []                # [rid, chain, bytes, steps left]
        used = 0
        batch = None
        dirty = False
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or waiting or active:
            t = now()
            while pending and results[pending[0]].arrival <= t:
                waiting.append(pending.popleft())
            # admission round: build the PT-MPOs of the next waiting requests,
            # then admit in arrival order while the handles fit the budget
            if waiting and len(active) < self.max_active:
                group = [rid for rid in list(waiting)[: self.max_admit] if rid not in built]
                if group:
                    tb = time.perf_counter()
                    new = self._build([(rid, requests[rid]) for rid in group])
                    dt_b = time.perf_counter() - tb
                    for rid in group:
                        built[rid] = new[rid]
                        results[rid].ptmpo_s = dt_b
                while waiting and len(active) < self.max_active and waiting[0] in built:
                    rid = waiting[0]
                    wl = requests[rid]
                    baths = self._baths(wl, built[rid])
                    need = B.workspace_bytes(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths,
                                             chi_max=wl["chi_max"], xi_max=wl["xi_max"], eps=wl["eps"],
                                             precision=self.precision)
                    if active and used + need > self.budget:
                        break
                    waiting.popleft()
                    ch = B.Chain(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths,
                                 chi_max=wl["chi_max"], xi_max=wl["xi_max"], eps=wl["eps"], precision=self.precision,
                                 stream=self.stream)
                    del built[rid]
                    active.append([rid, ch, need, int(wl["n_steps"])])
                    used += need
                    results[rid].admitted = now()
                    results[rid].bytes = need
                    dirty = True
            if not active:
                if pending:
                    time.sleep(max(0.0, results[pending[0]].arrival - now()))
                continue
            if dirty:
                if batch is not None:
                    batch.close()
                batch = B.Batch([a[1] for a in active])
                dirty = False
            batch.step(1)
            self._sync()
            finished = []
            for a in active:
                a[3] -= 1
                if a[3] == 0:
                    finished.append(a)
            if finished:
                batch.close()
                batch = None
                dirty = True
                for a in finished:
                    rid, ch = a[0], a[1]
                    n = requests[rid]["n_sites"]
                    sz, tr = ch.observe(np.arange(n, dtype=np.int32), np.array([SZ] * n))
                    r = results[rid]
                    r.sz, r.trace, r.done = sz, tr, now()
                    r.site_updates = n * int(requests[rid]["n_steps"])
                    ch.close()
                    used -= a[2]
                    active.remove(a)
                    if log:
                        log(f"request {rid} done at {r.done:.2f} s, latency {r.latency:.2f} s, "
                            f"{len(active)} active, {len(waiting)} waiting")
        if batch is not None:
            batch.close()
        return results


def run_alone(wl, precision=B.FP32_MIXED):
    """The same request stepped by itself (its own PT-MPO build, its own
    handle, pt_tebd_step): the reference for a result served in a mix."""
    keys, idx = _distinct_baths(wl)
    specs = []
    for key in keys:
        b = next(x for x in wl["baths"] if (x["alpha"], x["wc"], x["temperature"], x["k_cut"], x["cutoff"],
                                             x["coupling_op"].tobytes()) == key)
        specs.append(_bath_spec(b, wl["n_steps"]))
    pts = B.build_ptmpo_batch(specs, wl["dt"], wl["n_steps"], wl["baths"][0]["k_cut"], wl["eps_tempo"], wl["xi_max"])
    tensors = {key: pt["tensors"] for key, pt in zip(keys, pts)}
    baths = [{"site": b["site"], "tensors": tensors[keys[i]]} for b, i in zip(wl["baths"], idx)]
    ch = B.Chain(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths, chi_max=wl["chi_max"],
                 xi_max=wl["xi_max"], eps=wl["eps"], precision=precision)
    ch.step(int(wl["n_steps"]))
    n = wl["n_sites"]
    sz, tr = ch.observe(np.arange(n, dtype=np.int32), np.array([SZ] * n))
    ch.close()
    return sz, tr
