// Batched Hermitian eigensolver in double precision, one workgroup per
// problem.  Used for every Gram matrix of the bond update (the truncated
// SVDs of Appendix A.2 are computed from Gram matrices).
//
//  stage 1  Householder reduction A = Q T Q^H, T real symmetric tridiagonal
//           (reflector H_j = I - tau_j v_j v_j^H, H_j^H x = beta e_1)
//  stage 2  every eigenvalue of T by bisection on Sturm counts
//  stage 3  the selection rule (truncated-SVD rule of Appendix A.2, or a
//           numerical-rank rule) fixes how many leading eigenpairs are needed
//  stage 4  their eigenvectors of T by inverse iteration (pivoted LU of the
//           shifted tridiagonal), re-orthogonalised within clusters of
//           (near-)degenerate eigenvalues
//  stage 5  (separate kernel) back-transformation V = Q Z with the stored
//           reflectors
//  stage 6  (separate kernels) two passes of block classical Gram-Schmidt
//           of the columns of V in eigenvalue order, then the optional
//           column scaling
//
// Inverse iteration leaves eigenvectors whose mutual overlaps are about
// eps |lambda_0| / gap.  In a Gram matrix with a fast-decaying spectrum most
// gaps are tiny next to |lambda_0|, so overlaps of 1e-7 are common; the
// truncated SVDs built on these vectors reconstruct the two-site block only
// to that level.  Stage 6 removes the overlaps: one pass maps V to
// V (I - U), U the strictly upper part of V^H V, and renormalises the
// columns, which leaves overlaps of second order; the second pass brings
// them to rounding level.  Each column only loses components along the
// columns of larger eigenvalues, so the eigen-residuals stay at rounding
// level as well.
#pragma once

#include "device_common.h"
#include "gemm.h"

namespace ptt {

enum HeevRule : int {
  RULE_ALL = 0,    // every eigenpair with a positive eigenvalue
  RULE_EPS = 1,    // sqrt(eigenvalues) as singular values: eps rule only
  RULE_CAP = 2,    // eps rule + extra tail + chi_max cap + tie rule
  RULE_RANK = 3,   // numerical rank: lambda_k > rank_tol * lambda_0
  RULE_FULL = 4    // every eigenpair (the caller applies its own rule)
};

enum HeevScale : int { SCALE_NONE = 0, SCALE_INV_SQRT = 1, SCALE_SQRT = 2 };

struct HeevJob {
  double2* a;        // n x n Hermitian, row-major, leading dim lda (destroyed)
  int lda;
  const int* n_ptr;  // problem size on the device (0 = nothing to do)
  double* w;         // [>= n] eigenvalues, descending
  double2* refl;     // reflector storage [n_cap][n_cap]
  double* tri;       // [6 * n_cap] d, e, tau(re,im), misc
  double* work;      // inverse-iteration workspace [8 * n_cap * n_cap]
  double* z;         // tridiagonal eigenvectors [n_cap][n_cap] (row i, col k)
  int n_cap;
  int* nvec_out;     // number of eigenvectors selected
  int rule;
  double eps;        // RULE_EPS / RULE_CAP threshold
  int cap;           // RULE_CAP: chi_max
  const double* extra_tail;  // RULE_CAP: squared norm outside the spanned space (or null)
  double rank_tol;   // RULE_RANK
  double2* v;        // output eigenvectors, row-major n x nvec, leading dim ldv
  int ldv;
  int scale;         // HeevScale applied to column k with lambda_k
  int* status;       // sticky error word (bit 1: no convergence, bit 2: non-finite)
};

constexpr int HEEV_THREADS = 256;

// ------------------------------------------------------------- stage 1..4
__global__ void __launch_bounds__(HEEV_THREADS) heev_solve_kernel(const HeevJob* jobs) {
  const HeevJob& J = jobs[blockIdx.x];
  const int n = *J.n_ptr;
  const int tid = threadIdx.x;
  __shared__ double red[HEEV_THREADS / 64];
  __shared__ double2 sv[1024];  // current reflector v (n <= 1024)
  __shared__ double2 sw[1024];  // y then w
  __shared__ double2 s_tau;
  __shared__ double s_beta;
  __shared__ int s_nvec;
  if (n <= 0) return;  // nothing to do; *nvec_out is left as it is
  double2* A = J.a;
  const int lda = J.lda;
  double* dd = J.tri;              // diagonal of T
  double* ee = J.tri + J.n_cap;    // off-diagonal of T (ee[i] couples i, i+1)
  double2* taus = reinterpret_cast<double2*>(J.tri + 2 * J.n_cap);

  // -------- stage 1: reduction to tridiagonal form
  for (int j = 0; j + 1 < n; ++j) {
    const int m = n - j - 1;
    // column below the diagonal: x_i = A[j+1+i][j]
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += HEEV_THREADS) part += cabs2<double>(A[(size_t)(j + 1 + i) * lda + j]);
    const double sig2 = block_sum(part, red);
    if (tid == 0) {
      const double2 alpha = A[(size_t)(j + 1) * lda + j];
      double2 tau = mk<double>(0.0, 0.0);
      double beta = alpha.x;
      if (!(sig2 == 0.0 && alpha.y == 0.0)) {
        const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig2);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        tau = mk<double>((beta - alpha.x) / beta, -alpha.y / beta);
      }
      s_tau = tau;
      s_beta = beta;
      taus[j] = tau;
      ee[j] = beta;
    }
    __syncthreads();
    const double2 tau = s_tau;
    const double beta = s_beta;
    const bool active = !(tau.x == 0.0 && tau.y == 0.0);
    // v = x / (alpha - beta), v_0 = 1
    double2 scal = mk<double>(0.0, 0.0);
    {
      const double2 alpha = A[(size_t)(j + 1) * lda + j];
      const double2 den = mk<double>(alpha.x - beta, alpha.y);
      const double dn = den.x * den.x + den.y * den.y;
      if (active && dn > 0.0) scal = mk<double>(den.x / dn, -den.y / dn);
    }
    for (int i = tid; i < m; i += HEEV_THREADS) {
      double2 vi;
      if (i == 0) vi = mk<double>(1.0, 0.0);
      else vi = active ? cmul<double>(A[(size_t)(j + 1 + i) * lda + j], scal) : mk<double>(0.0, 0.0);
      sv[i] = vi;
      J.refl[(size_t)j * J.n_cap + i] = vi;
    }
    __syncthreads();
    if (active) {
      // y = tau * A22 v : one wave per row (coalesced along the row)
      const int lane = tid & 63, wid = tid >> 6;
      for (int r = wid; r < m; r += HEEV_THREADS / 64) {
        const double2* row = A + (size_t)(j + 1 + r) * lda + (j + 1);
        double2 acc = mk<double>(0.0, 0.0);
        for (int c = lane; c < m; c += 64) cfma<double>(acc, row[c], sv[c]);
        acc.x = warp_sum(acc.x);
        acc.y = warp_sum(acc.y);
        if (lane == 0) sw[r] = cmul<double>(tau, acc);
      }
      __syncthreads();
      // w = y - 1/2 Re(conj(tau) v^H y) v
      double2 p = mk<double>(0.0, 0.0);
      for (int i = tid; i < m; i += HEEV_THREADS) cfmaconj<double>(p, sv[i], sw[i]);
      const double vhy_re = block_sum(p.x, red);
      const double vhy_im = block_sum(p.y, red);
      const double half = 0.5 * (tau.x * vhy_re + tau.y * vhy_im);  // Re(conj(tau) vhy)
      __syncthreads();
      for (int i = tid; i < m; i += HEEV_THREADS) sw[i] = csub<double>(sw[i], cscale<double>(sv[i], half));
      __syncthreads();
      // A22 -= w v^H + v w^H
      for (int e = tid; e < m * m; e += HEEV_THREADS) {
        const int r = e / m, c = e - r * m;
        double2* dst = A + (size_t)(j + 1 + r) * lda + (j + 1 + c);
        double2 val = *dst;
        const double2 t1 = cmul<double>(sw[r], cconj<double>(sv[c]));
        const double2 t2 = cmul<double>(sv[r], cconj<double>(sw[c]));
        val.x -= t1.x + t2.x;
        val.y -= t1.y + t2.y;
        *dst = val;
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += HEEV_THREADS) dd[i] = A[(size_t)i * lda + i].x;
  if (tid == 0) ee[n - 1] = 0.0;
  __syncthreads();

  // -------- stage 2: eigenvalues by bisection (ascending index k)
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = fabs(dd[i]) + (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
    tnorm = fmax(tnorm, r);
  }
  const double glo = -tnorm, ghi = tnorm;
  const double pivmin = fmax(1e-300, 1e-290 * tnorm * tnorm);
  const double abstol = 2.2e-16 * tnorm * 0.5 + 1e-300;
  for (int k = tid; k < n; k += HEEV_THREADS) {
    double lo = glo - 1e-300, hi = ghi + 1e-300;
    for (int it = 0; it < 80; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (hi - lo <= fmax(abstol, 4.4e-16 * fmax(fabs(lo), fabs(hi)))) break;
      int cnt = 0;
      double q = dd[0] - mid;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      for (int i = 1; i < n; ++i) {
        q = dd[i] - mid - ee[i - 1] * ee[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
      }
      if (cnt > k) hi = mid;   // more than k eigenvalues below mid
      else lo = mid;
    }
    // store descending: position n-1-k
    J.w[n - 1 - k] = 0.5 * (lo + hi);
  }
  __syncthreads();

  // -------- stage 3: selection rule (thread 0)
  if (tid == 0) {
    const double* w = J.w;
    int nvec = 0;
    const double lam0 = w[0];
    if (J.rule == RULE_FULL) {
      nvec = n;
    } else if (J.rule == RULE_RANK) {
      while (nvec < n && w[nvec] > J.rank_tol * lam0 && w[nvec] > 0.0) ++nvec;
    } else {
      int npos = 0;
      while (npos < n && w[npos] > 0.0) ++npos;
      nvec = npos;
      if (J.rule != RULE_ALL && npos > 0) {
        const double extra = (J.rule == RULE_CAP && J.extra_tail) ? fmax(*J.extra_tail, 0.0) : 0.0;
        const double thr = J.eps * sqrt(lam0);
        // tail(c) = sqrt(extra + sum_{i >= c} w_i); smallest c with tail < thr
        double tail = extra;
        for (int i = npos - 1; i >= 1; --i) {
          tail += w[i];
          if (sqrt(tail) < thr) nvec = i;   // keeping i values leaves tail(i)
          else break;
        }
        if (J.rule == RULE_CAP && J.cap > 0 && nvec > J.cap) {
          nvec = J.cap;
          // tie rule on singular values: drop a split multiplet
          const double s0 = sqrt(lam0);
          while (nvec > 1 && sqrt(fmax(w[nvec - 1], 0.0)) - sqrt(fmax(w[nvec], 0.0)) < 1e-10 * s0) --nvec;
        }
      }
    }
    if (nvec < 1 && lam0 > 0.0) nvec = 1;
    if (!(lam0 == lam0) || isinf(lam0)) atomicOr(J.status, 4);
    s_nvec = nvec;
    *J.nvec_out = nvec;
  }
  __syncthreads();
  const int nvec = s_nvec;

  // -------- stage 4: inverse iteration, one thread per eigenvector
  // interleaved workspace: array a, row i, vector k at work[(a * n_cap + i) * n_cap + k]
  const int nc = J.n_cap;
  auto W = [&](int arr, int i, int k) -> double& { return J.work[((size_t)arr * nc + i) * nc + k]; };
  for (int k = tid; k < nvec; k += HEEV_THREADS) {
    const double lam = J.w[k];
    // shifted tridiagonal: dl = ee (sub), dg = dd - lam, du = ee (super), du2 = 0
    for (int i = 0; i < n; ++i) {
      W(0, i, k) = (i + 1 < n) ? ee[i] : 0.0;  // dl
      W(1, i, k) = dd[i] - lam;                // dg
      W(2, i, k) = (i + 1 < n) ? ee[i] : 0.0;  // du
      W(3, i, k) = 0.0;                        // du2
      W(4, i, k) = 0.0;                        // pivot flag
    }
    for (int i = 0; i + 1 < n; ++i) {
      const double di = W(1, i, k), li = W(0, i, k);
      if (fabs(di) >= fabs(li)) {
        const double f = (di != 0.0) ? li / di : 0.0;
        W(0, i, k) = f;
        W(1, i + 1, k) -= f * W(2, i, k);
        W(3, i, k) = 0.0;
        W(4, i, k) = 0.0;
      } else {
        const double f = di / li;
        W(1, i, k) = li;
        W(0, i, k) = f;
        const double tmp = W(2, i, k);
        W(2, i, k) = W(1, i + 1, k);
        W(1, i + 1, k) = tmp - f * W(1, i + 1, k);
        if (i + 2 < n) {
          W(3, i, k) = W(2, i + 1, k);
          W(2, i + 1, k) = -f * W(2, i + 1, k);
        }
        W(4, i, k) = 1.0;
      }
    }
    const double tiny = fmax(2.2e-16 * tnorm, 1e-300);
    for (int i = 0; i < n; ++i)
      if (fabs(W(1, i, k)) < tiny) W(1, i, k) = W(1, i, k) >= 0.0 ? tiny : -tiny;
    // start vector (deterministic pseudo-random, distinct per k)
    for (int i = 0; i < n; ++i) W(5, i, k) = u01(splitmix64(0x51ED2701ull * (k + 1) + i)) - 0.5;
    for (int it = 0; it < 3; ++it) {
      // forward (apply P and L)
      for (int i = 0; i + 1 < n; ++i) {
        if (W(4, i, k) != 0.0) {
          const double t = W(5, i, k);
          W(5, i, k) = W(5, i + 1, k);
          W(5, i + 1, k) = t;
        }
        W(5, i + 1, k) -= W(0, i, k) * W(5, i, k);
      }
      // backward (U)
      for (int i = n - 1; i >= 0; --i) {
        double s = W(5, i, k);
        if (i + 1 < n) s -= W(2, i, k) * W(6, i + 1, k);
        if (i + 2 < n) s -= W(3, i, k) * W(6, i + 2, k);
        W(6, i, k) = s / W(1, i, k);
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += W(6, i, k) * W(6, i, k);
      nrm = sqrt(nrm);
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int i = 0; i < n; ++i) W(5, i, k) = W(6, i, k) * inv;
    }
  }
  __syncthreads();
  // clusters of (near-)degenerate selected eigenvalues: orthogonalise each
  // member against its predecessors and iterate again (wave 0)
  if (tid < 64) {
    const int lane = tid;
    // clusters are formed among well-determined eigenvalues only
    // (lambda > 1e-12 |lambda_0|); below that the eigenvectors of a Gram
    // matrix are not resolved in double precision anyway
    const double gap_tol = 1e-10 * fmax(fabs(J.w[0]), 1e-300);
    const double floor_val = 1e-12 * fabs(J.w[0]);
    int nclu = 0;
    while (nclu < nvec && J.w[nclu] > floor_val) ++nclu;
    int start = 0;
    for (int k = 1; k <= nclu; ++k) {
      const bool brk = (k == nclu) || (fabs(J.w[k - 1] - J.w[k]) > gap_tol);
      if (!brk) continue;
      for (int j = start + 1; j < k; ++j) {
        for (int pass = 0; pass < 2; ++pass) {
          for (int p = start; p < j; ++p) {
            double dot = 0.0;
            for (int i = lane; i < n; i += 64) dot += W(5, i, p) * W(5, i, j);
            dot = warp_sum(dot);
            for (int i = lane; i < n; i += 64) W(5, i, j) -= dot * W(5, i, p);
          }
          // one more inverse-iteration solve with the member's own factors
          if (lane == 0) {
            for (int i = 0; i + 1 < n; ++i) {
              if (W(4, i, j) != 0.0) {
                const double t = W(5, i, j);
                W(5, i, j) = W(5, i + 1, j);
                W(5, i + 1, j) = t;
              }
              W(5, i + 1, j) -= W(0, i, j) * W(5, i, j);
            }
            for (int i = n - 1; i >= 0; --i) {
              double s = W(5, i, j);
              if (i + 1 < n) s -= W(2, i, j) * W(6, i + 1, j);
              if (i + 2 < n) s -= W(3, i, j) * W(6, i + 2, j);
              W(6, i, j) = s / W(1, i, j);
            }
            for (int i = 0; i < n; ++i) W(5, i, j) = W(6, i, j);
          }
          __builtin_amdgcn_wave_barrier();
          for (int p = start; p < j; ++p) {
            double dot = 0.0;
            for (int i = lane; i < n; i += 64) dot += W(5, i, p) * W(5, i, j);
            dot = warp_sum(dot);
            for (int i = lane; i < n; i += 64) W(5, i, j) -= dot * W(5, i, p);
          }
          double nrm = 0.0;
          for (int i = lane; i < n; i += 64) nrm += W(5, i, j) * W(5, i, j);
          nrm = warp_sum(nrm);
          const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
          for (int i = lane; i < n; i += 64) W(5, i, j) *= inv;
        }
      }
      start = k;
    }
  }
  __syncthreads();
  // vectors of eigenvalues below the resolution floor (and any later ones)
  // are undetermined individually; orthonormalise them against every
  // earlier vector (modified Gram-Schmidt, two passes, whole workgroup) so
  // the eigenvector matrix is unitary -- any orthonormal basis of that
  // subspace is equally valid.
  {
    __shared__ double dots[1024];
    __shared__ int s_j0;
    if (tid == 0) {
      const double floor_val = 1e-10 * fabs(J.w[0]);
      int j0 = 0;
      while (j0 < nvec && J.w[j0] > floor_val) ++j0;
      s_j0 = j0;
    }
    __syncthreads();
    for (int j = max(s_j0, 1); j < nvec; ++j) {
      for (int attempt = 0; attempt < 2; ++attempt) {
        for (int pass = 0; pass < 2; ++pass) {
          for (int i = tid; i < j; i += HEEV_THREADS) {
            double acc = 0.0;
            for (int r = 0; r < n; ++r) acc += W(5, r, i) * W(5, r, j);
            dots[i] = acc;
          }
          __syncthreads();
          for (int r = tid; r < n; r += HEEV_THREADS) {
            double acc = W(5, r, j);
            for (int i = 0; i < j; ++i) acc -= dots[i] * W(5, r, i);
            W(5, r, j) = acc;
          }
          __syncthreads();
        }
        double part = 0.0;
        for (int r = tid; r < n; r += HEEV_THREADS) part += W(5, r, j) * W(5, r, j);
        const double nrm = sqrt(block_sum(part, red));
        if (nrm > 1e-8 || attempt == 1) {
          const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
          for (int r = tid; r < n; r += HEEV_THREADS) W(5, r, j) *= inv;
          __syncthreads();
          break;
        }
        // nearly parallel to the earlier vectors: restart from a fresh vector
        for (int r = tid; r < n; r += HEEV_THREADS)
          W(5, r, j) = u01(splitmix64(0xC2B2AE3D27D4EB4Full * (j + 1) + r)) - 0.5;
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // publish Z (row i, column k)
  for (int e = tid; e < n * nvec; e += HEEV_THREADS) {
    const int i = e / nvec, k = e - i * nvec;
    J.z[(size_t)i * nc + k] = W(5, i, k);
  }
}

// --------------------------------------------------------------- stage 5
// V = Q Z for the selected columns; Q = H_0 H_1 ... H_{n-2}, so the
// reflectors are applied in the order H_{n-2}, ..., H_0.  Each workgroup
// keeps a chunk of HEEV_BT_COLS columns in LDS.
constexpr int HEEV_BT_COLS = 8;

__global__ void __launch_bounds__(HEEV_THREADS) heev_backtransform_kernel(const HeevJob* jobs) {
  const HeevJob& J = jobs[blockIdx.y];
  const int n = *J.n_ptr;
  const int nvec = (n > 0) ? *J.nvec_out : 0;
  const int c0 = blockIdx.x * HEEV_BT_COLS;
  if (c0 >= nvec) return;
  const int ncol = min(HEEV_BT_COLS, nvec - c0);
  extern __shared__ double2 zs[];  // [n][HEEV_BT_COLS]
  __shared__ double2 dots[HEEV_THREADS / 64][HEEV_BT_COLS];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nc = J.n_cap;
  for (int e = tid; e < n * HEEV_BT_COLS; e += HEEV_THREADS) {
    const int i = e / HEEV_BT_COLS, c = e - i * HEEV_BT_COLS;
    zs[e] = mk<double>(c < ncol ? J.z[(size_t)i * nc + c0 + c] : 0.0, 0.0);
  }
  const double2* taus = reinterpret_cast<const double2*>(J.tri + 2 * J.n_cap);
  __syncthreads();
  for (int j = n - 2; j >= 0; --j) {
    const double2 tau = taus[j];
    if (tau.x == 0.0 && tau.y == 0.0) continue;
    const int m = n - j - 1;
    const double2* v = J.refl + (size_t)j * nc;
    // s_c = sum_i conj(v_i) z[j+1+i][c]
    double2 part[HEEV_BT_COLS];
#pragma unroll
    for (int c = 0; c < HEEV_BT_COLS; ++c) part[c] = mk<double>(0.0, 0.0);
    for (int i = tid; i < m; i += HEEV_THREADS) {
      const double2 vi = v[i];
#pragma unroll
      for (int c = 0; c < HEEV_BT_COLS; ++c) cfmaconj<double>(part[c], vi, zs[(j + 1 + i) * HEEV_BT_COLS + c]);
    }
#pragma unroll
    for (int c = 0; c < HEEV_BT_COLS; ++c) {
      part[c].x = warp_sum(part[c].x);
      part[c].y = warp_sum(part[c].y);
    }
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < HEEV_BT_COLS; ++c) dots[wid][c] = part[c];
    __syncthreads();
    double2 s[HEEV_BT_COLS];
#pragma unroll
    for (int c = 0; c < HEEV_BT_COLS; ++c) {
      double2 acc = mk<double>(0.0, 0.0);
      for (int w2 = 0; w2 < HEEV_THREADS / 64; ++w2) acc = cadd<double>(acc, dots[w2][c]);
      s[c] = cmul<double>(tau, acc);
    }
    for (int i = tid; i < m; i += HEEV_THREADS) {
      const double2 vi = v[i];
#pragma unroll
      for (int c = 0; c < HEEV_BT_COLS; ++c) {
        double2& zz = zs[(j + 1 + i) * HEEV_BT_COLS + c];
        zz = csub<double>(zz, cmul<double>(s[c], vi));
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < n * ncol; e += HEEV_THREADS) {
    const int i = e / ncol, c = e - i * ncol;
    J.v[(size_t)i * J.ldv + c0 + c] = zs[i * HEEV_BT_COLS + c];
  }
}

// --------------------------------------------------------------- stage 6
// Scratch in the (by now free) inverse-iteration workspace, viewed as
// complex: G = V^H V at [0, n_cap^2), T = V (I - U) at [n_cap^2, 2 n_cap^2),
// both with leading dimension n_cap.
__device__ inline double2* orth_g(const HeevJob& J) { return reinterpret_cast<double2*>(J.work); }
__device__ inline double2* orth_t(const HeevJob& J) {
  return reinterpret_cast<double2*>(J.work) + (size_t)J.n_cap * J.n_cap;
}

// kind 0: G = V^H V (nvec x nvec);  kind 1: T = V M (n x nvec), M = I - U.
// grid (tiles_m, tiles_n, jobs)
__global__ void __launch_bounds__(GEMM_THREADS) heev_orth_gemm(const HeevJob* jobs, int kind) {
  __shared__ GemmSmem<double> sm;
  const HeevJob& J = jobs[blockIdx.z];
  const int n = *J.n_ptr;
  if (n <= 0) return;
  const int nvec = *J.nvec_out;
  if (nvec < 2) return;
  if (kind == 0)
    gemm_tile<double>(J.v, J.ldv, true, J.v, J.ldv, false, orth_g(J), J.n_cap, nvec, nvec, n,
                      mk<double>(1.0, 0.0), false, blockIdx.x, blockIdx.y, sm);
  else
    gemm_tile<double>(J.v, J.ldv, false, orth_g(J), J.n_cap, false, orth_t(J), J.n_cap, n, nvec, nvec,
                      mk<double>(1.0, 0.0), false, blockIdx.x, blockIdx.y, sm);
}

// G <- I - strictly_upper(G).  grid (blocks, jobs)
__global__ void heev_orth_mfix(const HeevJob* jobs) {
  const HeevJob& J = jobs[blockIdx.y];
  const int n = *J.n_ptr;
  if (n <= 0) return;
  const int nvec = *J.nvec_out;
  if (nvec < 2) return;
  double2* G = orth_g(J);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)nvec * nvec;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / nvec), j = (int)(e - (long long)i * nvec);
    double2& g = G[(size_t)i * J.n_cap + j];
    g = (i < j) ? mk<double>(-g.x, -g.y) : mk<double>(i == j ? 1.0 : 0.0, 0.0);
  }
}

// V <- T with unit columns (from_t), or V's own columns renormalised; the
// last call also applies the column scaling.  One thread per column.
// grid (ceil(n_cap / 256), jobs)
__global__ void heev_orth_norm(const HeevJob* jobs, int from_t, int final_pass) {
  const HeevJob& J = jobs[blockIdx.y];
  const int n = *J.n_ptr;
  if (n <= 0) return;
  const int nvec = *J.nvec_out;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nvec) return;
  const bool use_t = from_t && nvec >= 2;
  const double2* src = use_t ? orth_t(J) : J.v;
  const int lds = use_t ? J.n_cap : J.ldv;
  double acc = 0.0;
  for (int r = 0; r < n; ++r) acc += cabs2<double>(src[(size_t)r * lds + k]);
  double f = acc > 0.0 ? 1.0 / sqrt(acc) : 0.0;
  if (final_pass && J.scale != SCALE_NONE) {
    const double lam = fmax(J.w[k], 1e-300);
    f *= (J.scale == SCALE_INV_SQRT) ? 1.0 / sqrt(lam) : sqrt(lam);
  }
  for (int r = 0; r < n; ++r) J.v[(size_t)r * J.ldv + k] = cscale<double>(src[(size_t)r * lds + k], f);
}

}  // namespace ptt
