// Complex GEMM tile on the matrix cores (one 64 x 64 output tile per
// 256-thread workgroup), the counterpart of gemm_tile() in gemm.h:
//   C[m x n] = alpha * op(A)[m x k] * op(B)[k x n]   (+ C if accumulate)
// with op(X) = X or X^H, row-major operands of complex doubles in memory.
//
// The compute type CT is double (v_mfma_f64_16x16x4f64) or float
// (v_mfma_f32_16x16x4f32): operands are rounded to CT when they are staged
// into LDS and the products accumulate in CT, so the float form is the
// single-precision contraction of the mixed-precision path with the memory
// layout of the double one.  A complex product takes four real products
// (real-split form): Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
//
// Layout: LDS holds the real and imaginary planes of an A slice [BK][64]
// (k-major) and of a B slice [BK][64].  Wave w owns the 32 x 32 quarter
// (w / 2, w % 2) of the tile as 2 x 2 blocks of 16 x 16.  For one
// 16 x 16 x 4 step, lane l supplies A[row l % 16][k l / 16] and
// B[k l / 16][col l % 16]; its accumulator element r holds C[row][l % 16]
// with row = 4 (l / 16) + r for the single-precision instruction and
// row = l / 16 + 4 r for the double-precision one (both checked on gfx950
// against a host product).
#pragma once

#include "device_common.h"
#include "gemm.h"

namespace ptt {

typedef float mf_floatx4 __attribute__((ext_vector_type(4)));
typedef double mf_doublex4 __attribute__((ext_vector_type(4)));

template <typename CT> struct MfmaAcc;
template <> struct MfmaAcc<float> {
  using type = mf_floatx4;
  static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};
template <> struct MfmaAcc<double> {
  using type = mf_doublex4;
  static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};

__device__ inline mf_floatx4 mfma_16x16x4(float a, float b, mf_floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline mf_doublex4 mfma_16x16x4(double a, double b, mf_doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int MF_BK = 16;
constexpr int MF_LD = GEMM_BM * MF_BK / GEMM_THREADS;  // complex elements per operand each thread stages per slice

template <typename CT>
struct MfmaSmem {
  CT ar[MF_BK][GEMM_BM + 1], ai[MF_BK][GEMM_BM + 1];
  CT br[MF_BK][GEMM_BN + 1], bi[MF_BK][GEMM_BN + 1];
};

template <typename CT>
__device__ inline void gemm_tile_mfma(const double2* __restrict__ A, int lda, bool conjA,
                                      const double2* __restrict__ B, int ldb, bool conjB,
                                      double2* __restrict__ C, int ldc, int m, int n, int k,
                                      double2 alpha, bool accumulate, int tile_m, int tile_n,
                                      MfmaSmem<CT>& sm) {
  using acc_t = typename MfmaAcc<CT>::type;
  const int row0 = tile_m * GEMM_BM, col0 = tile_n * GEMM_BN;
  if (row0 >= m || col0 >= n) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cre[i][j][r] = 0;
        cim[i][j][r] = 0;
      }

  // staging coordinates: each operand is read along its row-major fast index
  int ar[MF_LD], ap[MF_LD], bc[MF_LD], bp[MF_LD];
#pragma unroll
  for (int t = 0; t < MF_LD; ++t) {
    const int e = tid + t * GEMM_THREADS;
    ar[t] = conjA ? (e & (GEMM_BM - 1)) : (e / MF_BK);
    ap[t] = conjA ? (e / GEMM_BM) : (e & (MF_BK - 1));
    bc[t] = conjB ? (e / MF_BK) : (e & (GEMM_BN - 1));
    bp[t] = conjB ? (e & (MF_BK - 1)) : (e / GEMM_BN);
  }
  double2 ra[MF_LD], rb[MF_LD];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < MF_LD; ++t) {
      const int gr = row0 + ar[t], gp = k0 + ap[t];
      ra[t] = mk<double>(0, 0);
      if (gr < m && gp < k) ra[t] = conjA ? cconj<double>(A[(size_t)gp * lda + gr]) : A[(size_t)gr * lda + gp];
      const int gc = col0 + bc[t], gq = k0 + bp[t];
      rb[t] = mk<double>(0, 0);
      if (gc < n && gq < k) rb[t] = conjB ? cconj<double>(B[(size_t)gc * ldb + gq]) : B[(size_t)gq * ldb + gc];
    }
  };
  load(0);
  const int li = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < k; k0 += MF_BK) {
#pragma unroll
    for (int t = 0; t < MF_LD; ++t) {
      sm.ar[ap[t]][ar[t]] = (CT)ra[t].x;
      sm.ai[ap[t]][ar[t]] = (CT)ra[t].y;
      sm.br[bp[t]][bc[t]] = (CT)rb[t].x;
      sm.bi[bp[t]][bc[t]] = (CT)rb[t].y;
    }
    __syncthreads();
    if (k0 + MF_BK < k) load(k0 + MF_BK);  // next slice in flight during the products
#pragma unroll
    for (int kk = 0; kk < MF_BK; kk += 4) {
      CT a_re[2], a_im[2], b_re[2], b_im[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a_re[i] = sm.ar[kk + lk][wr + 16 * i + li];
        a_im[i] = sm.ai[kk + lk][wr + 16 * i + li];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        b_re[j] = sm.br[kk + lk][wc + 16 * j + li];
        b_im[j] = sm.bi[kk + lk][wc + 16 * j + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = mfma_16x16x4(a_re[i], b_re[j], cre[i][j]);
          cre[i][j] = mfma_16x16x4(-a_im[i], b_im[j], cre[i][j]);
          cim[i][j] = mfma_16x16x4(a_re[i], b_im[j], cim[i][j]);
          cim[i][j] = mfma_16x16x4(a_im[i], b_re[j], cim[i][j]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr + 16 * i + MfmaAcc<CT>::row(lk, r);
        const int gc = col0 + wc + 16 * j + li;
        if (gr >= m || gc >= n) continue;
        const double2 acc = mk<double>((double)cre[i][j][r], (double)cim[i][j][r]);
        double2 v = cmul<double>(alpha, acc);
        double2* dst = C + (size_t)gr * ldc + gc;
        if (accumulate) v = cadd<double>(v, *dst);
        *dst = v;
      }
}

}  // namespace ptt
