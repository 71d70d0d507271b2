"""GPU tests of the continuous-batching request loop (serving.Server):
requests arriving while others are stepped are admitted under a device
memory budget and stepped together; every served result equals the same
request run alone (its own PT-MPO build, its own handle), because the
batched kernels run each chain's arithmetic unchanged and each PT-MPO is
built at its own request's length."""
import numpy as np
import pytest

from paper_2201_05529_amd import workloads as W
from tests.conftest import gpu_available
from tests.helpers import ensure_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_library()


def _requests(seed=7, n=7, xi_max=16, caps=(8, 16)):
    rng = np.random.default_rng(seed)
    out = []
    arrivals = [0.0, 0.0, 0.05, 0.1, 0.3, 0.3, 0.6][:n]
    for i in range(n):
        steps = int(rng.integers(6, 15))
        wl = W.random_xyz_chain(rng, f"req{i}", 3, 5, caps, steps, dt=0.05, k_cut=3, xi_max=xi_max)
        wl["arrival_s"] = arrivals[i]
        out.append(wl)
    return out


def _peak_bytes(results):
    # admissions and completions in time order (a completion before an
    # admission at the same instant: the loop frees before it admits)
    events = sorted([(r.admitted, 1, r.bytes) for r in results] + [(r.done, 0, -r.bytes) for r in results])
    cur = best = 0
    for _, _, b in events:
        cur += b
        best = max(best, cur)
    return best


@pytest.mark.parametrize("precision", [0, 1])
def test_served_results_equal_alone(precision):
    from paper_2201_05529_amd import binding as B
    from paper_2201_05529_amd import serving as S
    reqs = _requests()
    print(f"serving precision={precision}", flush=True)
    # a budget that holds about three handles at once
    sizes = []
    for wl in reqs:
        pts = B.build_ptmpo_batch([{"alpha": wl["baths"][0]["alpha"], "wc": 4.0,
                                    "temperature": wl["baths"][0]["temperature"], "coupling_op": W.SZ}],
                                  wl["dt"], wl["n_steps"], 3, wl["eps_tempo"], wl["xi_max"])
        baths = [{"site": b["site"], "tensors": pts[0]["tensors"]} for b in wl["baths"]]
        sizes.append(B.workspace_bytes(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths,
                                       chi_max=wl["chi_max"], xi_max=wl["xi_max"], eps=wl["eps"], precision=precision))
    budget = int(3.2 * max(sizes))
    srv = S.Server(budget, precision=precision, max_active=8, max_admit=4)
    res = srv.run(reqs, realtime=True)
    assert all(r.done is not None for r in res)
    assert all(r.admitted >= r.arrival - 1e-9 for r in res)
    assert _peak_bytes(res) <= budget
    # requests waited for memory, and others were admitted while some ran
    assert any(r.admitted > r.arrival + 1e-3 for r in res)
    worst = 0.0
    for wl, r in zip(reqs, res):
        sz, tr = S.run_alone(wl, precision=precision)
        worst = max(worst, float(np.abs(r.sz - sz).max()), abs(r.trace - tr))
    print(f"  largest difference served vs alone: {worst:.1e}; latencies "
          + " ".join(f"{r.latency:.2f}" for r in res), flush=True)
    assert worst <= 1e-12


def test_served_results_match_the_oracle():
    # the served FP64 results against the oracle stepped with the oracle's
    # PT-MPO builder (the builders agree to about eps_TEMPO).  One bath per
    # request and a chi cap of 64 that these chains do not reach (at most 41)
    # keep every truncation decision at the eps rule: where the cap binds in
    # the middle of a slowly decaying spectrum, the GPU's leading subspace of
    # D (a randomized range finder) is less accurate than a dense SVD and
    # the trajectories part at ~1e-6 per step
    from oracle import pt_tebd as opt
    from oracle.build import problem_from_workload
    from paper_2201_05529_amd import serving as S
    reqs = _requests(seed=11, n=4, xi_max=64, caps=(64,))
    for wl in reqs:
        wl["eps_tempo"] = 1e-10
        wl["baths"] = wl["baths"][:1]
    res = S.Server(1 << 40, precision=0).run(reqs, realtime=False)
    worst = 0.0
    for wl, r in zip(reqs, res):
        prob, _ = problem_from_workload(wl)
        eng = opt.Engine(prob)
        eng.step(int(wl["n_steps"]))
        ref = np.array([eng.expectation(s, W.SZ) for s in range(wl["n_sites"])])
        worst = max(worst, float(np.abs(r.sz - ref).max()))
    print(f"served vs oracle: {worst:.1e}", flush=True)
    assert worst < 1e-6
