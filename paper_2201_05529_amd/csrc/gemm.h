// Tiled complex GEMM tile routine (one 64 x 64 output tile per 256-thread
// workgroup), used by every contraction kernel of the bond update.
//   C[m x n] = alpha * op(A)[m x k] * op(B)[k x n]   (+ C if accumulate)
// op(X) is X or its conjugate transpose; all matrices are row-major with
// leading dimension = row stride.  Dimensions are run-time values read from
// device memory by the caller, so tiles outside [m, n] return at once.
#pragma once

#include "device_common.h"

namespace ptt {

constexpr int GEMM_BM = 64, GEMM_BN = 64, GEMM_BK = 8, GEMM_THREADS = 256;

template <typename T>
struct GemmSmem {
  cx<T> a[GEMM_BK][GEMM_BM + 1];
  cx<T> b[GEMM_BK][GEMM_BN + 1];
};

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

  for (int k0 = 0; k0 < k; k0 += GEMM_BK) {
    // A tile: BM x BK elements, 2 per thread
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int e = tid + t * GEMM_THREADS;
      int r, p;
      if (conjA) { r = e & 63; p = e >> 6; }   // coalesced along r
      else { p = e & 7; r = e >> 3; }          // coalesced along p
      const int gr = row0 + r, gp = k0 + p;
      cx<T> v = mk<T>(0, 0);
      if (gr < m && gp < k) v = conjA ? cconj<T>(A[(size_t)gp * lda + gr]) : A[(size_t)gr * lda + gp];
      sm.a[p][r] = v;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int e = tid + t * GEMM_THREADS;
      int c, p;
      if (conjB) { p = e & 7; c = e >> 3; }
      else { c = e & 63; p = e >> 6; }
      const int gc = col0 + c, gp = k0 + p;
      cx<T> v = mk<T>(0, 0);
      if (gc < n && gp < k) v = conjB ? cconj<T>(B[(size_t)gc * ldb + gp]) : B[(size_t)gp * ldb + gc];
      sm.b[p][c] = v;
    }
    __syncthreads();
#pragma unroll
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
