"""GPU parity for the model variants the method covers beyond sigma^z
coupling: baths coupled through non-diagonal operators (sigma^y, sigma^x:
the PT-MPO tensors are dense in the system index, Sec. III.A), GKSL
dissipators in the chain propagators (Appendix A.1), and both at once.
The library is fed the oracle's PT-MPO tensors; observables within 1e-6 of
the oracle (FP64) and 1e-4 (FP32-mixed)."""
import numpy as np
import pytest

from oracle import pt_tebd as opt
from paper_2201_05529_amd import workloads as W
from tests.conftest import gpu_available
from tests.helpers import ensure_library, library_chain, oracle_problem, run_both

pytestmark = pytest.mark.gpu
SX, SY, SZ = W.SX, W.SY, W.SZ
SM = np.array([[0, 0], [1, 0]], dtype=np.complex128)   # sigma^- = |down><up| in the (up, down) basis
TOL = {0: 1e-6, 1: 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_library()


def _chain(n, baths, lindblad=None, steps=10):
    j = [(1.1, 0.8, 0.6), (0.9, 1.2, 0.7), (1.3, 0.6, 1.0)]
    bonds = [W.xyz_bond(*j[b % 3]) for b in range(n - 1)]
    rho0 = [W.UP] + [W.DOWN] * (n - 1)
    wl = W.make_chain("variant", n, bonds, [0.3] * n, rho0, dt=0.1, n_steps=steps, baths=baths, chi_max=64,
                      xi_max=64, eps=1e-10, eps_tempo=1e-12)
    wl["lindblad"] = lindblad
    return wl


def _ops(n):
    return [(s, SZ) for s in range(n)] + [(s, SX) for s in range(n)]


def _check(wl, precision, steps=10):
    g, o, gt, ot, ch, _ = run_both(wl, steps, _ops(wl["n_sites"]), precision=precision)
    ch.close()
    err, terr = float(np.abs(g - o).max()), float(np.abs(gt - ot).max())
    print(f"  max |d<op>| {err:.1e}  max |d Tr| {terr:.1e}", flush=True)
    assert err < TOL[precision] and terr < TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_coupling_baths(precision):
    # sigma^y on site 0 and sigma^x on site 2: the influence factors are
    # diagonal only in each coupling operator's eigenbasis, so the tensors
    # handed to the chain are dense 4 x 4 in the Liouville index
    print(f"dense coupling precision={precision}", flush=True)
    wl = _chain(3, [W.bath(0, 0.1, 4.0, 1.0, 3, coupling=SY), W.bath(2, 0.08, 4.0, 0.7, 3, coupling=SX)])
    prob = oracle_problem(wl, n_steps=10)
    assert all(p.ndim == 4 for b in prob.baths for p in b["tensors"])
    _check(wl, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_gksl_dissipators(precision):
    # amplitude damping on every site and dephasing on site 1, with a
    # sigma^z bath on site 0
    print(f"GKSL precision={precision}", flush=True)
    n = 4
    lind = [[np.sqrt(0.2) * SM] for _ in range(n)]
    lind[1].append(np.sqrt(0.1) * SZ)
    wl = _chain(n, [W.bath(0, 0.1, 4.0, 1.0, 3)], lindblad=lind)
    _check(wl, precision)


def test_gksl_and_dense_coupling_together():
    print("GKSL + dense coupling", flush=True)
    lind = [[np.sqrt(0.15) * SM], [], [np.sqrt(0.05) * SZ]]
    wl = _chain(3, [W.bath(1, 0.12, 4.0, 1.5, 3, coupling=SY)], lindblad=lind)
    _check(wl, 0)
