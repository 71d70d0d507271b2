"""GPU tests of batches (pt_tebd_batch_*): chains of different lengths, bond
caps and PT-MPOs advanced together, one launch per kernel of a sublayer
across chains, one time step captured in a HIP graph.  Every chain's result
is bit-identical to the same chain stepped alone: the batched kernels run
the same per-item arithmetic, only the grids differ."""
import os

import numpy as np
import pytest

from paper_2201_05529_amd import workloads as W
from tests.conftest import gpu_available
from tests.helpers import ensure_library, library_chain, oracle_problem

pytestmark = pytest.mark.gpu
SZ, SX = W.SZ, W.SX


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_library()


SPECS = [(410, 3, (0,), 16), (411, 5, (0, 4), 32), (412, 4, (1, 2), 64), (413, 6, (0, 3, 5), 24), (414, 2, (1,), 8)]


def _problems(steps):
    wls, probs = [], []
    for seed, n, sites, chi in SPECS:
        wl = W.random_small_chain(seed, n, with_bath_sites=sites, k_cut=3, eps=1e-8, xi_max=32, chi_max=chi)
        wls.append(wl)
        probs.append(oracle_problem(wl, n_steps=steps))
    return wls, probs


def _observe(ch, n):
    v, tr = ch.observe(range(n), np.array([SZ] * n))
    v2, _ = ch.observe(range(n), np.array([SX] * n))
    return np.concatenate([v, v2, [tr]])


@pytest.mark.parametrize("graph,precision", [(True, 0), (False, 0), (True, 1)])
def test_batch_matches_chains_alone(graph, precision):
    import torch
    from paper_2201_05529_amd import binding as B
    steps = 6
    wls, probs = _problems(steps + 1)
    alone = []
    for wl, prob in zip(wls, probs):
        ch = library_chain(wl, prob, precision=precision)
        out = []
        for _ in range(steps):
            ch.step(1)
            out.append(_observe(ch, wl["n_sites"]))
        alone.append(np.array(out))
        ch.close()
    stream = torch.cuda.Stream()
    chains = [library_chain(wl, prob, precision=precision, stream=stream) for wl, prob in zip(wls, probs)]
    os.environ["PT_TEBD_GRAPH"] = "1" if graph else "0"
    try:
        batch = B.Batch(chains)
    finally:
        os.environ.pop("PT_TEBD_GRAPH", None)
    got = [[] for _ in chains]
    for _ in range(steps):
        batch.step(1)
        for i, (ch, wl) in enumerate(zip(chains, wls)):
            got[i].append(_observe(ch, wl["n_sites"]))
    for a, g in zip(alone, got):
        assert np.array_equal(a, np.array(g))
    assert all(ch.current_step == steps for ch in chains)
    batch.close()


def test_batch_with_chains_at_different_steps():
    # chains enter the batch at different steps (as requests do in serving);
    # the device step counters follow each chain
    import torch
    from paper_2201_05529_amd import binding as B
    wls, probs = _problems(8)
    stream = torch.cuda.Stream()
    ref = []
    for k, (wl, prob) in enumerate(zip(wls, probs)):
        ch = library_chain(wl, prob)
        ch.step(k % 3 + 4)
        ref.append(_observe(ch, wl["n_sites"]))
        ch.close()
    chains = [library_chain(wl, prob, stream=stream) for wl, prob in zip(wls, probs)]
    for k, ch in enumerate(chains):
        ch.step(k % 3)            # alone first
    batch = B.Batch(chains)
    batch.step(2)
    batch.step(2)                 # the captured graph replayed
    for k, (ch, wl) in enumerate(zip(chains, wls)):
        assert ch.current_step == k % 3 + 4
        assert np.array_equal(ref[k], _observe(ch, wl["n_sites"]))
    batch.close()


def test_batch_rejects_mixed_streams_and_past_the_end():
    import torch
    from paper_2201_05529_amd import binding as B
    wls, probs = _problems(3)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = library_chain(wls[0], probs[0], stream=s1)
    b = library_chain(wls[1], probs[1], stream=s2)
    with pytest.raises(B.PtTebdError):
        B.Batch([a, b])
    c = library_chain(wls[2], probs[2], stream=s1)
    batch = B.Batch([a, c])
    with pytest.raises(B.PtTebdError) as e:
        batch.step(4)             # the PT-MPOs have 3 steps
    assert e.value.status == -6
    assert a.current_step == 0 and c.current_step == 0
    batch.close()


def test_step_many_is_a_batch():
    import torch
    from paper_2201_05529_amd import binding as B
    wls, probs = _problems(4)
    stream = torch.cuda.Stream()
    chains = [library_chain(wl, prob, stream=stream) for wl, prob in zip(wls, probs)]
    B.step_many(chains, 3)
    for wl, prob, ch in zip(wls, probs, chains):
        solo = library_chain(wl, prob)
        solo.step(3)
        assert np.array_equal(_observe(solo, wl["n_sites"]), _observe(ch, wl["n_sites"]))
