// Second orthonormalisation pass of the range finder by Cholesky QR.
//
// The first pass (eigenvalues of the Gram matrix, scaled by lambda^-1/2, with
// rank revelation) leaves a basis Y whose Gram matrix G = Y^H Y is the
// identity up to rounding amplified by the conditioning of the sketch.  For
// such a G the eigenvalue route is the slowest possible input (one cluster of
// n eigenvalues), while G = R^H R (R upper triangular with a positive
// diagonal) is cheap and exact: Y R^-1 has orthonormal columns spanning the
// same space.  The kernel writes W = R^-1 (upper triangular, zero below the
// diagonal) into the n x n block of vk; the caller then forms Y W with the
// same product it uses after an eigenvalue pass.  G itself is left intact.
//
// A job is declined, and the eigenvalue pass runs for it instead, when n is
// above CHOL_NMAX or a pivot is not a finite number above CHOL_PIVOT_FLOOR
// times the largest diagonal entry of G: the kernel stores n in the
// fallback dimension for such a job and 0 otherwise.
//
// Layout: one workgroup of CHOL_THREADS threads per job.  Thread t owns
// column c = t mod CHOL_NMAX and the rows r = t / CHOL_NMAX + 8 m
// (m = 0..15) of that column, in registers, for the whole factorisation and
// inversion.  Each elimination step broadcasts one row (and, during the
// inversion, one column) through double-buffered LDS, so a step costs one
// barrier.
#pragma once

#include "bond_kernels.h"

namespace ptt {

constexpr int CHOL_NMAX = 128;
constexpr int CHOL_THREADS = 1024;
constexpr int CHOL_ROWS = CHOL_THREADS / CHOL_NMAX;   // row groups (8)
constexpr int CHOL_PER = CHOL_NMAX / CHOL_ROWS;       // rows per thread (16)
constexpr double CHOL_PIVOT_FLOOR = 1e-6;

// grid (items); dims[size_dim] is the Gram size, gk (ld k_cap) the Gram
// matrix; the declined size goes to dims[fb_dim]
__global__ void __launch_bounds__(CHOL_THREADS) k_chol_inv(const BondJob* jobs, int size_dim, int fb_dim) {
  const BondJob& J = jobs[blockIdx.x];
  int* D = J.dims;
  const int t = threadIdx.x;
  const int n = D[D_RF] != 0 ? D[size_dim] : 0;
  if (n <= 0 || n > CHOL_NMAX) {
    if (t == 0) D[fb_dim] = n > 0 ? n : 0;
    return;
  }
  const int ld = J.k_cap;
  const int c = t % CHOL_NMAX, rg = t / CHOL_NMAX;
  __shared__ double2 rbuf[2][CHOL_NMAX];
  __shared__ double2 cbuf[2][CHOL_NMAX];
  __shared__ double dinv[CHOL_NMAX];
  __shared__ double piv[2][4];  // p, 1/p, sqrt(p), 1/sqrt(p) of the current step
  __shared__ double red[CHOL_THREADS / 64];

  // upper triangle of G into registers; largest diagonal entry
  double2 a[CHOL_PER];
  double dloc = 0.0;
#pragma unroll
  for (int m = 0; m < CHOL_PER; ++m) {
    const int i = rg + CHOL_ROWS * m;
    a[m] = (i <= c && c < n) ? J.gk[(long long)i * ld + c] : mk<double>(0.0, 0.0);
    if (i == c && c < n) dloc = a[m].x;
  }
  {
    double v = dloc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((t & 63) == 0) red[t >> 6] = v;
  }
  __syncthreads();
  double dmax = red[0];
  for (int w = 1; w < CHOL_THREADS / 64; ++w) dmax = fmax(dmax, red[w]);
  const double floor_piv = CHOL_PIVOT_FLOOR * dmax;

  // G = R^H R, right-looking: step k publishes row k of the reduced matrix,
  // then every owner of an element (i, j), k < i <= j, subtracts
  // conj(A_ki) A_kj / A_kk and the owners of row k scale it to R_k.
  bool fail = !(dmax > 0.0) || !(dmax < INFINITY);
  for (int k = 0; k < n && !fail; ++k) {
    double2* buf = rbuf[k & 1];
    if (rg == (k % CHOL_ROWS) && c >= k && c < n) {
#pragma unroll
      for (int m = 0; m < CHOL_PER; ++m)
        if (m == k / CHOL_ROWS) {
          buf[c] = a[m];
          if (c == k) {  // the pivot's owner does the divisions once for everyone
            const double p = a[m].x, r = sqrt(p);
            piv[k & 1][0] = p;
            piv[k & 1][1] = 1.0 / p;
            piv[k & 1][2] = r;
            piv[k & 1][3] = 1.0 / r;
            dinv[k] = 1.0 / r;
          }
        }
    }
    __syncthreads();
    const double p = piv[k & 1][0];
    if (!(p > floor_piv) || !(p < INFINITY)) { fail = true; break; }  // same value in every thread
    const double ip = piv[k & 1][1], rkk = piv[k & 1][2], irk = piv[k & 1][3];
    if (c > k && c < n) {
      const double2 bc = buf[c];
#pragma unroll
      for (int m = 0; m < CHOL_PER; ++m) {
        const int i = rg + CHOL_ROWS * m;
        if (i > k && i <= c) {
          const double2 bi = buf[i];
          // a -= conj(bi) * bc / p
          double2 s = mk<double>(0.0, 0.0);
          cfmaconj<double>(s, bi, bc);
          a[m].x = fma(-s.x, ip, a[m].x);
          a[m].y = fma(-s.y, ip, a[m].y);
        } else if (i == k) {
          a[m] = cscale<double>(a[m], irk);
        }
      }
    } else if (c == k) {
#pragma unroll
      for (int m = 0; m < CHOL_PER; ++m)
        if (rg + CHOL_ROWS * m == k) a[m] = mk<double>(rkk, 0.0);
    }
  }
  if (fail) {
    if (t == 0) D[fb_dim] = n;
    return;
  }
  __syncthreads();  // dinv complete

  // W = R^-1 in place, right-looking from the last column: with B = I
  // initially, step k (n-1 down to 0) takes row k of W as B_k / R_kk and
  // subtracts R_ik W_k from every row i < k.  Column k of R is read out (and
  // replaced by column k of B) in the same step, which is its last use.
  for (int k = n - 1; k >= 0; --k) {
    double2* cb = cbuf[k & 1];
    double2* rb = rbuf[k & 1];
    const double dk = dinv[k];
    if (c == k) {
#pragma unroll
      for (int m = 0; m < CHOL_PER; ++m) {
        const int i = rg + CHOL_ROWS * m;
        if (i < k) {
          cb[i] = a[m];
          a[m] = mk<double>(0.0, 0.0);
        } else if (i == k) {
          a[m] = mk<double>(1.0, 0.0);
        }
      }
    }
    if (rg == (k % CHOL_ROWS) && c >= k && c < n) {
#pragma unroll
      for (int m = 0; m < CHOL_PER; ++m)
        if (m == k / CHOL_ROWS) {
          a[m] = cscale<double>(a[m], dk);
          rb[c] = a[m];
        }
    }
    __syncthreads();
    if (c >= k && c < n) {
      const double2 wc = rb[c];
#pragma unroll
      for (int m = 0; m < CHOL_PER; ++m) {
        const int i = rg + CHOL_ROWS * m;
        if (i < k) {
          const double2 ri = cb[i];
          a[m].x = fma(-ri.x, wc.x, a[m].x);
          a[m].x = fma(ri.y, wc.y, a[m].x);
          a[m].y = fma(-ri.x, wc.y, a[m].y);
          a[m].y = fma(-ri.y, wc.x, a[m].y);
        }
      }
    }
  }

  // W (upper triangular) into vk, zeros below the diagonal
  if (c < n) {
#pragma unroll
    for (int m = 0; m < CHOL_PER; ++m) {
      const int i = rg + CHOL_ROWS * m;
      if (i < n) J.vk[(long long)i * ld + c] = (i <= c) ? a[m] : mk<double>(0.0, 0.0);
    }
  }
  if (t == 0) D[fb_dim] = 0;
}

}  // namespace ptt
