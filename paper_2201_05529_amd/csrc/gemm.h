// Tiled complex GEMM tile routine (one 64 x 64 output tile per 256-thread
// workgroup), used by every contraction kernel of the bond update.
//   C[m x n] = alpha * op(A)[m x k] * op(B)[k x n]   (+ C if accumulate)
// op(X) is X or its conjugate transpose; all matrices are row-major with
// leading dimension = row stride.  Dimensions are run-time values read from
// device memory by the caller, so tiles outside [m, n] return at once.
#pragma once

#include "device_common.h"

namespace ptt {

constexpr int GEMM_BM = 64, GEMM_BN = 64, GEMM_BK = 16, GEMM_THREADS = 256;
constexpr int GEMM_LD = GEMM_BM * GEMM_BK / GEMM_THREADS;  // elements of A (and of B) each thread loads per k-step

template <typename T>
struct GemmSmem {
  cx<T> a[GEMM_BK][GEMM_BM + 1];
  cx<T> b[GEMM_BK][GEMM_BN + 1];
};

// The next k-slice is loaded into registers while the current one is
// multiplied out of LDS, so global latency overlaps the arithmetic; two
// barriers per slice of GEMM_BK.
template <typename T>
__device__ inline void gemm_tile(const cx<T>* __restrict__ A, int lda, bool conjA,
                                 const cx<T>* __restrict__ B, int ldb, bool conjB,
                                 cx<T>* __restrict__ C, int ldc, int m, int n, int k,
                                 cx<T> alpha, bool accumulate, int tile_m, int tile_n,
                                 GemmSmem<T>& sm) {
  const int row0 = tile_m * GEMM_BM, col0 = tile_n * GEMM_BN;
  if (row0 >= m || col0 >= n) return;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  cx<T> acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk<T>(0, 0);

  // element e = tid + t * GEMM_THREADS of a slice; each operand is read
  // along its row-major fast index (coalesced)
  int ar[GEMM_LD], ap[GEMM_LD], bc[GEMM_LD], bp[GEMM_LD];
#pragma unroll
  for (int t = 0; t < GEMM_LD; ++t) {
    const int e = tid + t * GEMM_THREADS;
    ar[t] = conjA ? (e & (GEMM_BM - 1)) : (e / GEMM_BK);
    ap[t] = conjA ? (e / GEMM_BM) : (e & (GEMM_BK - 1));
    bc[t] = conjB ? (e / GEMM_BK) : (e & (GEMM_BN - 1));
    bp[t] = conjB ? (e & (GEMM_BK - 1)) : (e / GEMM_BN);
  }
  cx<T> ra[GEMM_LD], rb[GEMM_LD];
#pragma unroll
  for (int t = 0; t < GEMM_LD; ++t) {
    const int gr = row0 + ar[t], gp = ap[t];
    ra[t] = mk<T>(0, 0);
    if (gr < m && gp < k) ra[t] = conjA ? cconj<T>(A[(size_t)gp * lda + gr]) : A[(size_t)gr * lda + gp];
    const int gc = col0 + bc[t], gq = bp[t];
    rb[t] = mk<T>(0, 0);
    if (gc < n && gq < k) rb[t] = conjB ? cconj<T>(B[(size_t)gc * ldb + gq]) : B[(size_t)gq * ldb + gc];
  }
  for (int k0 = 0; k0 < k; k0 += GEMM_BK) {
#pragma unroll
    for (int t = 0; t < GEMM_LD; ++t) {
      sm.a[ap[t]][ar[t]] = ra[t];
      sm.b[bp[t]][bc[t]] = rb[t];
    }
    __syncthreads();
    const int k1 = k0 + GEMM_BK;
    if (k1 < k) {
#pragma unroll
      for (int t = 0; t < GEMM_LD; ++t) {
        const int gr = row0 + ar[t], gp = k1 + ap[t];
        ra[t] = mk<T>(0, 0);
        if (gr < m && gp < k) ra[t] = conjA ? cconj<T>(A[(size_t)gp * lda + gr]) : A[(size_t)gr * lda + gp];
        const int gc = col0 + bc[t], gq = k1 + bp[t];
        rb[t] = mk<T>(0, 0);
        if (gc < n && gq < k) rb[t] = conjB ? cconj<T>(B[(size_t)gc * ldb + gq]) : B[(size_t)gq * ldb + gc];
      }
    }
    // two k-steps per iteration: full unrolling hoists every LDS load and
    // spills; two keep the accumulators and operands in registers
#pragma unroll 2
    for (int p = 0; p < GEMM_BK; ++p) {
      cx<T> av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sm.a[p][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sm.b[p][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfma<T>(acc[i][j], av[i], bv[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gr = row0 + ty + 16 * i;
    if (gr >= m) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gc = col0 + tx + 16 * j;
      if (gc >= n) continue;
      cx<T> v = cmul<T>(alpha, acc[i][j]);
      cx<T>* dst = C + (size_t)gr * ldc + gc;
      if (accumulate) v = cadd<T>(v, *dst);
      *dst = v;
    }
  }
}

}  // namespace ptt
