// Host-side double-precision helpers of the PT-TEBD library: chain
// propagators, bath influence coefficients, PT-MPO construction.  None of
// this is on the per-step hot path; it runs once per handle.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace ptt {

using cplx = std::complex<double>;

// Row-major dense complex matrix helpers.
std::vector<cplx> matmul(int n, int k, int m, const cplx* a, const cplx* b);

// exp(A) for a small dense matrix by scaling and squaring of a Taylor
// polynomial carried to double-precision convergence.
std::vector<cplx> expm(int n, const cplx* a);

// Hermitian eigensolver (Householder reduction to a real tridiagonal matrix,
// implicit-shift QL iteration with eigenvector accumulation).  Eigenvalues
// ascending in w[n]; eigenvector k is column k of v (row-major n x n).
// Returns false if the QL iteration does not converge.
bool heev(int n, const cplx* a, double* w, cplx* v);

// Chain propagators (Appendix A.1).  h_site [N][d][d], h_bond [N-1][d2][d2]
// natural order, lindblad [N][n_l][d][d] or null.  Returns, per bond, the
// site-major d^4 x d^4 gate exp(L^{K'} tau) with tau = dt/2 on 1-based odd
// bonds and dt/4 on 1-based even bonds.  For N = 1, returns the single-site
// half-step propagator exp(L^S dt/2) (d^2 x d^2) instead.
std::vector<std::vector<cplx>> chain_gates(int n_sites, int d, double dt, const cplx* h_site,
                                           const cplx* h_bond, int n_lind, const cplx* lindblad);

// Influence coefficients eta_Delta, Delta = 0..k_cut, for the piecewise-
// constant-path discretisation of a Gaussian bath (see pt_bath_eta).
bool bath_eta(double alpha, double wc, int cutoff_kind, double temperature, double dt, int k_cut,
              std::vector<cplx>& eta, std::string& err);

// PT-MPO of a bath with coupling eigenvalues sigma (d of them): tensors
// P_k[e][e'][x] in the coupling eigenbasis, bond dims [M+1].
bool build_ptmpo(const std::vector<cplx>& eta, const std::vector<double>& sigma, int n_steps,
                 double eps, int xi_max, std::vector<std::vector<cplx>>& tensors,
                 std::vector<int>& dims, std::string& err);

// Cap vectors by backward recursion (trace the output, maximally mixed
// input).  tensors[k] is P_{k+1} laid out [e][e'][d2] (diagonal) or
// [e][e'][d2][d2] (dense).
std::vector<std::vector<cplx>> caps_backward(const std::vector<std::vector<cplx>>& tensors,
                                             const std::vector<int>& dims, int d, bool diagonal);

}  // namespace ptt
