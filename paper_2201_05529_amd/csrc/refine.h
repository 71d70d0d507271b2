// Block refinement of Gram-based singular values.
//
// A Gram eigensolver resolves singular values only to ~1e-8 of the largest
// (eigenvalues are squared singular values), which is where the truncation
// rule of Appendix A.2 decides with eps ~ 1e-7.  After the first solve, the
// vectors (columns of B V, or rows of U^H B) whose norms are below tau times
// the largest form a block; the Gram matrix of that block alone is solved
// again and the block is rotated by its eigenvectors, so the block's
// singular values are now resolved relative to the block's own scale.  The
// step repeats on the next block (levels), and the singular values are the
// vector norms after the last level.
#pragma once

#include "device_common.h"
#include "gemm.h"
#include "heev.h"

namespace ptt {

struct RefineJob {
  double2* P;
  int ldp;                         // leading dim of P (if ldp_ptr is null)
  const int* ldp_ptr;              // run-time leading dim of P (or null)
  int cols;                        // 1: vectors are the columns of P (len x n); 0: rows (n x len)
  const int* side_ptr;             // if set: cols = (*side_ptr == side_cols)
  int side_cols;
  const int* len_cols;             // vector length when cols == 1
  const int* len_rows;             // vector length when cols == 0
  const int* n_ptr;                // number of vectors
  double2* V; int ldv;             // matrix whose columns follow the vectors (nv x n)
  const int* nv_ptr;               // rows of V
  double* s;                       // norms [n]
  int* blk;                        // [2]: block start p, block size m (0: nothing left)
  double2* G; int ldg;             // block Gram matrix (m x m)
  double2* W; int ldw;             // block eigenvectors (m x m)
  double2* TP; int ldtp;           // rotated P block
  double2* TV; int ldtv;           // rotated V block
};

__device__ inline int ref_cols(const RefineJob& R) { return R.side_ptr ? (*R.side_ptr == R.side_cols) : R.cols; }
__device__ inline int ref_len(const RefineJob& R) { return ref_cols(R) ? *R.len_cols : *R.len_rows; }
__device__ inline int ref_ldp(const RefineJob& R) { return R.ldp_ptr ? *R.ldp_ptr : R.ldp; }

// norms of every vector, one wave per vector.  grid (blocks, jobs)
__global__ void k_ref_norms(const RefineJob* jobs) {
  const RefineJob& R = jobs[blockIdx.y];
  const int n = *R.n_ptr, len = ref_len(R), ldp = ref_ldp(R), cols = ref_cols(R);
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int wid = blockIdx.x * nw + (threadIdx.x >> 6), stride = gridDim.x * nw;
  const long long si = cols ? 1 : ldp, se = cols ? ldp : 1;
  for (int i = wid; i < n; i += stride) {
    double acc = 0.0;
    for (int e = lane; e < len; e += 64) acc += cabs2<double>(R.P[(long long)i * si + (long long)e * se]);
    acc = warp_sum(acc);
    if (lane == 0) R.s[i] = sqrt(acc);
  }
}

// choose the block of the next level: first index after the previous block
// start whose norm is below tau times the previous block's leading norm.
// level 0 starts from the whole set.  One thread per job.
__global__ void k_ref_select(const RefineJob* jobs, int n_jobs, double tau, int level) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_jobs) return;
  const RefineJob& R = jobs[j];
  const int n = *R.n_ptr;
  int start = 0;
  if (level > 0) {
    if (R.blk[1] == 0) return;  // nothing was refined at the previous level
    start = R.blk[0];
  }
  int p = n;
  if (n > 0) {
    const double ref = R.s[start];
    for (int i = start + 1; i < n; ++i)
      if (R.s[i] < tau * ref) { p = i; break; }
  }
  R.blk[0] = p;
  R.blk[1] = (n - p >= 2 && p < n) ? n - p : 0;
}

enum RefKind : int { RK_GRAM = 0, RK_ROTP, RK_ROTV };

__device__ inline bool ref_args(const RefineJob& R, int kind, const double2*& A, int& lda, bool& ca,
                                const double2*& B, int& ldb, bool& cb, double2*& C, int& ldc, int& m, int& n,
                                int& k) {
  const int p = R.blk[0], bm = R.blk[1];
  if (bm <= 0) return false;
  const int len = ref_len(R), ldp = ref_ldp(R), cols = ref_cols(R);
  switch (kind) {
    case RK_GRAM:
      if (cols) {  // G = P[:, p:]^H P[:, p:]
        A = R.P + p; lda = ldp; ca = true; B = R.P + p; ldb = ldp; cb = false;
      } else {     // G = P[p:, :] P[p:, :]^H
        A = R.P + (long long)p * ldp; lda = ldp; ca = false; B = A; ldb = ldp; cb = true;
      }
      C = R.G; ldc = R.ldg; m = bm; n = bm; k = len;
      return true;
    case RK_ROTP:
      if (cols) {  // TP (len x bm) = P[:, p:] W
        A = R.P + p; lda = ldp; ca = false; B = R.W; ldb = R.ldw; cb = false;
        C = R.TP; ldc = R.ldtp; m = len; n = bm; k = bm;
      } else {     // TP (bm x len) = W^H P[p:, :]
        A = R.W; lda = R.ldw; ca = true; B = R.P + (long long)p * ldp; ldb = ldp; cb = false;
        C = R.TP; ldc = R.ldtp; m = bm; n = len; k = bm;
      }
      return true;
    case RK_ROTV:    // TV (nv x bm) = V[:, p:] W
      A = R.V + p; lda = R.ldv; ca = false; B = R.W; ldb = R.ldw; cb = false;
      C = R.TV; ldc = R.ldtv; m = *R.nv_ptr; n = bm; k = bm;
      return true;
  }
  return false;
}

// grid (tiles_m, tiles_n, jobs)
__global__ void __launch_bounds__(GEMM_THREADS) k_ref_gemm(const RefineJob* jobs, int kind) {
  __shared__ GemmSmem<double> sm;
  const RefineJob& R = jobs[blockIdx.z];
  const double2 *A, *B;
  double2* C;
  int lda, ldb, ldc, m, n, k;
  bool ca, cb;
  if (!ref_args(R, kind, A, lda, ca, B, ldb, cb, C, ldc, m, n, k)) return;
  if (m <= 0 || n <= 0) return;
  gemm_tile<double>(A, lda, ca, B, ldb, cb, C, ldc, m, n, k, mk<double>(1.0, 0.0), false, blockIdx.x,
                    blockIdx.y, sm);
}

// write the rotated blocks back.  grid (blocks, jobs)
__global__ void k_ref_copy(const RefineJob* jobs) {
  const RefineJob& R = jobs[blockIdx.y];
  const int p = R.blk[0], bm = R.blk[1];
  if (bm <= 0) return;
  const int len = ref_len(R), nv = *R.nv_ptr, ldp = ref_ldp(R), cols = ref_cols(R);
  const long long np = (long long)len * bm, nvv = (long long)nv * bm;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < np + nvv;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < np) {
      if (cols) {
        const int e = (int)(idx / bm), c = (int)(idx - (long long)e * bm);
        R.P[(long long)e * ldp + p + c] = R.TP[(long long)e * R.ldtp + c];
      } else {
        const int r = (int)(idx / len), e = (int)(idx - (long long)r * len);
        R.P[(long long)(p + r) * ldp + e] = R.TP[(long long)r * R.ldtp + e];
      }
    } else {
      const long long j = idx - np;
      const int r = (int)(j / bm), c = (int)(j - (long long)r * bm);
      R.V[(long long)r * R.ldv + p + c] = R.TV[(long long)r * R.ldtv + c];
    }
  }
}

}  // namespace ptt
