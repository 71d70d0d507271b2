/*
 * pt_tebd_testing.h -- test-only entry points of libpt_tebd.so.
 *
 * They run one device kernel family of the PT-TEBD path on caller data so
 * that it can be checked in isolation.  They allocate device memory with
 * hipMalloc (not for use under graph capture) and synchronise.
 */
#ifndef PT_TEBD_TESTING_H
#define PT_TEBD_TESTING_H

#include "pt_tebd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Hermitian eigensolver of the truncated SVDs (Householder tridiagonal
 * reduction, bisection, inverse iteration, back-transformation) on one n x n
 * Hermitian matrix a (complex, row-major, n <= 1024).  rule: 0 every positive
 * eigenvalue, 1 the eps rule on sqrt(eigenvalues), 2 the eps rule plus the
 * cap, 3 numerical rank (lambda_k > eps * lambda_0), 4 every eigenpair.  Returns the eigenvalues
 * in w[n] (descending), the selected eigenvectors in v (complex, row-major
 * n x n, column k = vector k) and their number in *nvec. */
pt_tebd_status pt_test_heev(int32_t n, const double* a, int32_t rule, double eps, int32_t cap,
                            double* w, double* v, int32_t* nvec);

/* pt_test_heev that also returns the real tridiagonal matrix T = Q^H a Q of
 * the first stage (tri[0..n): diagonal, tri[n..2n): off-diagonal, entry i
 * coupling rows i and i + 1) and the eigenvectors of T before the
 * back-transformation (z, row-major n x n; column k pairs with w[k] for the
 * selected columns k < *nvec). */
pt_tebd_status pt_test_heev_tridiagonal(int32_t n, const double* a, int32_t rule, double eps, int32_t cap,
                                        double* w, double* v, int32_t* nvec, double* tri, double* z);

/* Stage times of the eigensolver on one matrix (rule as pt_test_heev),
 * averaged over reps runs on fresh copies of a: stage_ms[0..5] the
 * tridiagonal reduction, the shifted factorisation, the eigenvalues, the
 * selection rule, the twisted eigenvectors and the cluster pass (device
 * wall clock inside the kernels; the factorisation's time includes the
 * launch gap between the reduction kernel and the stage 2-4 kernel),
 * stage_ms[6] the two kernels together and stage_ms[7] the
 * back-transformation plus the two orthonormalisation passes (HIP events).
 * stage_ms holds 9 doubles ([8] is zero). */
pt_tebd_status pt_test_heev_profile(int32_t n, const double* a, int32_t rule, double eps, int32_t reps,
                                    double* stage_ms);

#ifdef __cplusplus
}
#endif

#endif /* PT_TEBD_TESTING_H */
