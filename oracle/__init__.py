"""Plain FP64 CPU oracle for PT-TEBD (arXiv 2201.05529).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (the HIP library and its Python binding) never
imports, links or calls anything here, and nothing here imports the product.

Everything is complex128 / float64, written step by step in the paper's
order with NumPy/SciPy primitives (``numpy.linalg.svd``, ``scipy.linalg.expm``,
``scipy.integrate.quad``) and no blocking or fusion.

Modules
-------
liouville     vectorisation, super-operators, two-site index permutation
              (Appendix A.1: the calculation is carried out in Liouville space)
bath          spectral density, bath correlation function and the discretised
              influence coefficients eta_Delta (Appendix B.1)
ptmpo         influence-functional factors, exact history-form PT-MPO,
              TEMPO-style window-compressed PT-MPO, cap tensors (Sec. II.A,
              Appendix A.1 and A.3)
pt_tebd       augmented MPS and the PT-TEBD step: two-site update (c-h),
              PT absorption (i-j), observables via caps (k-l), two-time
              correlations (Appendix A.2-A.4)
brute         dense full-Liouville-space references used to pin pt_tebd
closed_forms  analytically solvable special cases used to pin everything

Pinning status of each function is stated in its module docstring; every
function here is pinned by a ``-m "not gpu"`` test against something other
than itself (closed forms, brute force, invariants).
"""
