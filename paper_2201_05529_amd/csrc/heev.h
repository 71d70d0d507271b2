// Batched Hermitian eigensolver in double precision, one workgroup per
// problem.  Used for every Gram matrix of the bond update (the truncated
// SVDs of Appendix A.2 are computed from Gram matrices).
//
//  stage 1  Householder reduction A = Q T Q^H, T real symmetric tridiagonal
//           (reflector H_j = I - tau_j v_j v_j^H, H_j^H x = beta e_1)
//  stage 2  T + delta I = L D L^T with D > 0 (delta a few ulps of |T|, more
//           if needed, so the factorisation exists)
//  stage 3  every eigenvalue of L D L^T by multisection on qd negcounts, to
//           high relative accuracy; then the selection rule (truncated-SVD
//           rule of Appendix A.2, or a numerical-rank rule) fixes how many
//           leading eigenpairs are needed
//  stage 4  their eigenvectors of T from twisted factorisations (one O(n)
//           solve per vector); clusters of numerically equal eigenvalues
//           get random starts, inverse iteration and Gram-Schmidt; the
//           unresolved tail (eigenvalues at the rounding level) gets an
//           orthonormal basis of the complement by Householder QR
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

constexpr int HEEV_THREADS = 256;          // back-transformation kernel
constexpr int HEEV_SOLVE_THREADS = 1024;   // solve kernel (stages 1-4)

// Number of eigenvalues of L D L^T below sigma (L unit lower bidiagonal with
// subdiagonal l, D = diag(d) > 0), by the differential stationary qd
// transform: s_0 = -sigma, D+_i = d_i + s_i, s_{i+1} = l_i^2 d_i s_i / D+_i
// - sigma.  The count is the number of negative D+_i (Sylvester).  Computed
// from the factors, the count resolves every eigenvalue to high relative
// accuracy (a factored positive definite tridiagonal is a relatively robust
// representation).
__device__ inline int ldl_negcount(const double* d, const double* lld, int n, double sigma, double pivmin) {
  int cnt = 0;
  double s = -sigma;
  for (int i = 0; i + 1 < n; ++i) {
    double dp = d[i] + s;
    if (fabs(dp) < pivmin) dp = -pivmin;
    cnt += dp < 0.0;
    s = lld[i] * (s / dp) - sigma;
  }
  double dp = d[n - 1] + s;
  if (fabs(dp) < pivmin) dp = -pivmin;
  cnt += dp < 0.0;
  return cnt;
}

// ------------------------------------------------------------- stage 1..4
__global__ void __launch_bounds__(HEEV_SOLVE_THREADS) heev_solve_kernel(const HeevJob* jobs) {
  constexpr int NT = HEEV_SOLVE_THREADS;
  const HeevJob& J = jobs[blockIdx.x];
  const int n = *J.n_ptr;
  if (n <= 0) return;  // nothing to do; *nvec_out is left as it is
  const int tid = threadIdx.x;
  __shared__ double buf[8192];     // stage 1: two v, w, partial sums; later: d, l, l d, l^2 d, mu, tau
  __shared__ double red[NT / 64];
  __shared__ double2 s_tau;
  __shared__ double s_beta, s_delta, s_tnorm;
  __shared__ int s_nvec, s_ok;
  double2* A = J.a;
  const int lda = J.lda;
  const int nc = J.n_cap;
  double* dd = J.tri;              // diagonal of T
  double* ee = J.tri + nc;         // off-diagonal of T (ee[i] couples i, i+1)
  double2* taus = reinterpret_cast<double2*>(J.tri + 2 * nc);

  // -------- stage 1: reduction to real tridiagonal form, T = Q^H A Q.
  // Both triangles of the trailing block are kept.  The rank-2 update of
  // step j is not applied at once: step j+1 first forms its own row from the
  // pending update, then one fused pass over the trailing block applies the
  // pending update and accumulates the next matrix-vector product, so every
  // element is read and written once per step.  Each pass is coalesced
  // along rows (thread c of a row group owns column c).
  {
    double2* vbuf0 = reinterpret_cast<double2*>(buf);
    double2* vbuf1 = vbuf0 + 1024;
    double2* sw = vbuf1 + 1024;   // pending w, then the new w
    double2* part = sw + 1024;
    double2* vp = vbuf0;          // pending v (offset j at step j)
    double2* vc = vbuf1;          // current v
    bool pending = false;
    for (int j = 0; j + 1 < n; ++j) {
      const int m = n - j - 1, off = j + 1;
      // (a) row j of the updated matrix: x = conj(row) below the diagonal
      for (int i = tid; i < m; i += NT) {
        double2 val = A[(size_t)j * lda + off + i];
        if (pending) {
          const double2 t1 = cmul<double>(sw[0], cconj<double>(vp[i + 1]));
          const double2 t2 = cmul<double>(vp[0], cconj<double>(sw[i + 1]));
          val.x -= t1.x + t2.x;
          val.y -= t1.y + t2.y;
        }
        vc[i] = cconj<double>(val);
      }
      if (tid == 0) {
        double a = A[(size_t)j * lda + j].x;
        if (pending) a -= 2.0 * (sw[0].x * vp[0].x + sw[0].y * vp[0].y);
        dd[j] = a;
      }
      __syncthreads();
      double p = 0.0;
      for (int i = 1 + tid; i < m; i += NT) p += cabs2<double>(vc[i]);
      const double sig2 = block_sum(p, red);
      if (tid == 0) {
        const double2 alpha = vc[0];
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
      double2 scal = mk<double>(0.0, 0.0);
      {
        const double2 alpha = vc[0];
        const double2 den = mk<double>(alpha.x - beta, alpha.y);
        const double dn = den.x * den.x + den.y * den.y;
        if (active && dn > 0.0) scal = mk<double>(den.x / dn, -den.y / dn);
      }
      __syncthreads();  // everyone has read vc[0]
      for (int i = tid; i < m; i += NT) {
        double2 vi;
        if (i == 0) vi = mk<double>(1.0, 0.0);
        else vi = active ? cmul<double>(vc[i], scal) : mk<double>(0.0, 0.0);
        vc[i] = vi;
        J.refl[(size_t)j * nc + i] = vi;
      }
      __syncthreads();
      // (b) fused pass: A22 -= pending update; part = conj(A22)^T v
      const int groups = max(1, NT / m);
      const int c = tid % m, g = tid / m;
      if (g < groups) {
        double2 acc = mk<double>(0.0, 0.0);
        if (pending) {
          const double2 vpc = cconj<double>(vp[c + 1]), wpc = cconj<double>(sw[c + 1]);
#pragma unroll 4
          for (int r = g; r < m; r += groups) {
            double2* dst = A + (size_t)(off + r) * lda + off + c;
            double2 val = *dst;
            const double2 t1 = cmul<double>(sw[r + 1], vpc);
            const double2 t2 = cmul<double>(vp[r + 1], wpc);
            val.x -= t1.x + t2.x;
            val.y -= t1.y + t2.y;
            *dst = val;
            cfmaconj<double>(acc, val, vc[r]);
          }
        } else {
#pragma unroll 4
          for (int r = g; r < m; r += groups) cfmaconj<double>(acc, A[(size_t)(off + r) * lda + off + c], vc[r]);
        }
        part[g * m + c] = acc;
      }
      __syncthreads();
      // (c) w = tau y - 1/2 Re(conj(tau) v^H tau y) v becomes the pending update
      double2 pv = mk<double>(0.0, 0.0);
      double2 y = mk<double>(0.0, 0.0);
      if (tid < m) {
        for (int q = 0; q < groups; ++q) y = cadd<double>(y, part[q * m + tid]);
        y = cmul<double>(tau, y);
        cfmaconj<double>(pv, vc[tid], y);
      }
      const double vhy_re = block_sum(pv.x, red);
      const double vhy_im = block_sum(pv.y, red);
      const double half = 0.5 * (tau.x * vhy_re + tau.y * vhy_im);
      if (tid < m) sw[tid] = csub<double>(y, cscale<double>(vc[tid], half));
      __syncthreads();
      double2* t = vp;
      vp = vc;
      vc = t;
      pending = true;
    }
    if (tid == 0) {
      double a = A[(size_t)(n - 1) * lda + (n - 1)].x;
      if (pending) a -= 2.0 * (sw[0].x * vp[0].x + sw[0].y * vp[0].y);
      dd[n - 1] = a;
      ee[n - 1] = 0.0;
    }
  }
  __syncthreads();

  // -------- stage 2: T + delta I = L D L^T with D > 0
  double* d = buf;
  double* l = buf + 1024;
  double* ld = buf + 2048;
  double* lld = buf + 3072;
  double* mu = buf + 4096;
  if (tid == 0) {
    double tn = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = fabs(dd[i]) + (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
      tn = fmax(tn, r);
    }
    s_tnorm = tn;
    int ok = 0;
    double delta = fmax(8.0 * n * 2.2e-16 * tn, 1e-300);
    if (tn > 0.0) {
      for (int attempt = 0; attempt < 64 && !ok; ++attempt) {
        ok = 1;
        double di = dd[0] + delta;
        for (int i = 0; i < n; ++i) {
          if (!(di > 1e-300 * fmax(tn, 1.0))) { ok = 0; break; }
          d[i] = di;
          if (i + 1 < n) {
            const double li = ee[i] / di;
            l[i] = li;
            ld[i] = li * di;
            lld[i] = li * li * di;
            di = (dd[i + 1] + delta) - li * ee[i];
          }
        }
        if (!ok) delta = fmin(delta * 8.0, 4.0 * tn);
      }
    }
    s_delta = delta;
    s_ok = ok;
  }
  __syncthreads();
  const double tnorm = s_tnorm;
  const double delta = s_delta;
  if (!s_ok) {
    // zero matrix (or a factorisation that never became definite): every
    // eigenvalue is taken as zero and Z = I
    for (int i = tid; i < n; i += NT) {
      J.w[i] = 0.0;
      mu[i] = 0.0;
    }
    if (tnorm > 0.0 && tid == 0) atomicOr(J.status, 1);
  } else {
    // -------- stage 3: eigenvalues of L D L^T by multisection, four
    // threads per eigenvalue, geometric splits (relative accuracy)
    const double pivmin = 1e-290 * fmax(1.0, tnorm * tnorm);
    const int q = tid & 3;
    for (int k0 = 0; k0 < n; k0 += NT / 4) {
      const int k = k0 + (tid >> 2);
      double lo = 1e-300 * (tnorm + delta), hi = 1.01 * (tnorm + delta) + 1e-300;
      if (k < n) {
        for (int it = 0; it < 120; ++it) {
          if (hi - lo <= 4.4e-16 * hi) break;
          const bool geo = lo > 0.0 && hi > 4.0 * lo;
          const double f = (q + 1) * 0.2;
          const double x = geo ? lo * exp(f * log(hi / lo)) : lo + f * (hi - lo);
          const int cnt = ldl_negcount(d, lld, n, x, pivmin);
          // gather the four (x, cnt) pairs of this quad
          double nlo = lo, nhi = hi;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double xr = __shfl(x, ((threadIdx.x & 63) & ~3) + r, 64);
            const int cr = __shfl(cnt, ((threadIdx.x & 63) & ~3) + r, 64);
            if (cr <= k) nlo = fmax(nlo, xr);
            else nhi = fmin(nhi, xr);
          }
          lo = nlo;
          hi = nhi;
        }
      }
      if (k < n && q == 0) {
        const double m_k = 0.5 * (lo + hi);
        mu[k] = m_k;
        J.w[n - 1 - k] = m_k - delta;
      }
    }
  }
  __syncthreads();

  // -------- stage 3b: selection rule (thread 0)
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

  // -------- stage 4: eigenvectors of T by twisted factorisations of
  // L D L^T - mu I (one thread per vector).  Top-down: D+_i = d_i + s_i,
  // l+_i = l_i d_i / D+_i; bottom-up: D-_i = l_{i-1}^2 d_{i-1} + p_i,
  // u-_i = l_i d_i / D-_{i+1}, p_i = d_i p_{i+1} / D-_{i+1} - mu.  The twist
  // index r minimises |gamma_r| = |s_r + p_r + mu|; z_r = 1 and
  // z_i = -l+_i z_{i+1} above r, z_{i+1} = -u-_i z_i below.  With mu accurate
  // to high relative accuracy the vector's error is O(n eps) / relgap, so
  // vectors of distinct eigenvalues come out orthogonal without any
  // reorthogonalisation.  Per-vector arrays interleave by vector index.
  auto W = [&](int arr, int i, int k) -> double& { return J.work[((size_t)arr * nc + i) * nc + k]; };
  auto Z = [&](int i, int k) -> double& { return J.z[(size_t)i * nc + k]; };
  if (!s_ok) {
    for (int e = tid; e < n * nvec; e += NT) {
      const int i = e / nvec, k = e - i * nvec;
      Z(i, k) = (i == k) ? 1.0 : 0.0;
    }
    return;
  }
  const double pivmin = 1e-290 * fmax(1.0, tnorm * tnorm);
  // eigenvalues within the rounding level of the reduction (lambda <= delta,
  // a few n eps |T|) are not resolved: their vectors are any orthonormal
  // basis of the complement of the resolved ones (stage 4c).  They form a
  // tail of the descending order.
  int nres = 0;
  while (nres < nvec && J.w[nres] > delta) ++nres;
  for (int k = tid; k < nres; k += NT) {
    const double m_k = mu[n - 1 - k];
    // top-down (stationary)
    double s = -m_k;
    for (int i = 0; i + 1 < n; ++i) {
      W(1, i, k) = s;
      double dp = d[i] + s;
      if (fabs(dp) < pivmin) dp = dp < 0.0 ? -pivmin : pivmin;
      W(0, i, k) = ld[i] / dp;
      s = lld[i] * (s / dp) - m_k;
    }
    W(1, n - 1, k) = s;
    // bottom-up (progressive) with the twist index
    double p = d[n - 1] - m_k;
    double gmin = fabs(W(1, n - 1, k) + p + m_k);
    int r = n - 1;
    for (int i = n - 2; i >= 0; --i) {
      double dm = lld[i] + p;
      if (fabs(dm) < pivmin) dm = dm < 0.0 ? -pivmin : pivmin;
      const double t = d[i] / dm;
      W(2, i, k) = l[i] * t;
      p = p * t - m_k;
      const double g = fabs(W(1, i, k) + p + m_k);
      if (g < gmin) { gmin = g; r = i; }
    }
    // solve
    double z = 1.0, nrm = 1.0;
    Z(r, k) = 1.0;
    for (int i = r - 1; i >= 0; --i) {
      z = -W(0, i, k) * z;
      Z(i, k) = z;
      nrm += z * z;
    }
    z = 1.0;
    for (int i = r; i + 1 < n; ++i) {
      z = -W(2, i, k) * z;
      Z(i + 1, k) = z;
      nrm += z * z;
    }
    const double inv = (nrm > 0.0 && nrm < 1e300) ? 1.0 / sqrt(nrm) : 0.0;
    if (inv > 0.0) {
      for (int i = 0; i < n; ++i) Z(i, k) *= inv;
    } else {  // overflow: fall back to the unit vector at the twist index
      for (int i = 0; i < n; ++i) Z(i, k) = (i == r) ? 1.0 : 0.0;
    }
  }
  __syncthreads();

  // -------- stage 4b: clusters of numerically equal eigenvalues (relative
  // gap below 1e-9).  Twisted vectors of equal mu coincide, so every member
  // after the first restarts from a seeded random vector, takes two
  // inverse-iteration solves with its own top-down factors, and is
  // orthogonalised against the earlier members (one wave per cluster).
  {
    const double rgap = 1e-9;
    auto same = [&](int a, int b) {  // a, b descending-order indices
      const double ma = mu[n - 1 - a], mb = mu[n - 1 - b];
      return fabs(ma - mb) <= rgap * fmax(fabs(ma), fabs(mb));
    };
    // pivots of the (nearly) singular shifted matrix are floored at
    // eps |T|, as in inverse iteration: the solve then amplifies the
    // eigenspace without overflowing
    const double pfloor = fmax(2.2e-16 * tnorm, pivmin);
    // members: k with k > 0 and same(k - 1, k)
    for (int k = tid; k < nres; k += NT) {
      if (k == 0 || !same(k - 1, k)) continue;
      const double m_k = mu[n - 1 - k];
      // top-down factors of L D L^T - mu I with floored pivots: W(0) = l+,
      // W(1) = D+
      double s = -m_k;
      for (int i = 0; i < n; ++i) {
        double dp = d[i] + s;
        if (fabs(dp) < pfloor) dp = dp < 0.0 ? -pfloor : pfloor;
        W(1, i, k) = dp;
        if (i + 1 < n) {
          W(0, i, k) = ld[i] / dp;
          s = lld[i] * (s / dp) - m_k;
        }
      }
      for (int i = 0; i < n; ++i) Z(i, k) = u01(splitmix64(0xA24BAED4963EE407ull * (k + 1) + i)) - 0.5;
      for (int it = 0; it < 2; ++it) {
        // (L+ D+ L+^T) y = z: forward with L+, divide by D+, backward with L+^T
        for (int i = 0; i + 1 < n; ++i) Z(i + 1, k) -= W(0, i, k) * Z(i, k);
        for (int i = 0; i < n; ++i) Z(i, k) /= W(1, i, k);
        for (int i = n - 2; i >= 0; --i) Z(i, k) -= W(0, i, k) * Z(i + 1, k);
        double nr = 0.0;
        for (int i = 0; i < n; ++i) nr += Z(i, k) * Z(i, k);
        const double inv = (nr > 0.0 && nr < 1e300) ? 1.0 / sqrt(nr) : 0.0;
        for (int i = 0; i < n; ++i) Z(i, k) *= inv;
      }
    }
    __syncthreads();
    const int lane = tid & 63, wid = tid >> 6;
    // cluster starts, handed out round-robin to the waves
    int cl = 0;
    for (int k = 0; k < nres; ++k) {
      if (k > 0 && same(k - 1, k)) continue;  // not a start
      int e = k + 1;
      while (e < nres && same(e - 1, e)) ++e;
      if (e - k >= 2 && (cl++ % (NT / 64)) == wid) {
        for (int j = k + 1; j < e; ++j) {
          for (int pass = 0; pass < 2; ++pass) {
            for (int q2 = k; q2 < j; ++q2) {
              double dot = 0.0;
              for (int i = lane; i < n; i += 64) dot += Z(i, q2) * Z(i, j);
              dot = warp_sum(dot);
              for (int i = lane; i < n; i += 64) Z(i, j) -= dot * Z(i, q2);
            }
            double nr = 0.0;
            for (int i = lane; i < n; i += 64) nr += Z(i, j) * Z(i, j);
            nr = warp_sum(nr);
            const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
            for (int i = lane; i < n; i += 64) Z(i, j) *= inv;
          }
        }
      }
    }
  }
  if (nres >= nvec) return;
  __syncthreads();

  // -------- stage 4c: unresolved tail.  Householder QR of a copy of the
  // resolved vectors Z_h (n x h, orthonormal): H_{h-1} ... H_0 Z_h = [R; 0].
  // Then Q = H_0 ... H_{h-1} and its columns h, h+1, ... are an orthonormal
  // basis of the complement; column c = Q e_c is built by one thread
  // applying the reflectors to e_c.  Reflector j is kept in W(3, i >= j, j),
  // the copy of Z_h in W(4), tau_j in LDS.
  {
    double* rtau = buf + 5120;  // <= 1024 reflectors
    const int h = nres;
    for (int e = tid; e < n * h; e += NT) {
      const int i = e / h, c = e - i * h;
      W(4, i, c) = Z(i, c);
    }
    __syncthreads();
    for (int j = 0; j < h; ++j) {
      double part = 0.0;
      for (int i = j + 1 + tid; i < n; i += NT) part += W(4, i, j) * W(4, i, j);
      const double sig2 = block_sum(part, red);
      if (tid == 0) {
        const double alpha = W(4, j, j);
        double tau = 0.0, beta = alpha;
        if (sig2 > 0.0) {
          const double nrm = sqrt(alpha * alpha + sig2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
        }
        rtau[j] = tau;
        s_beta = (tau != 0.0) ? 1.0 / (alpha - beta) : 0.0;
      }
      __syncthreads();
      const double scl = s_beta;
      const double tau = rtau[j];
      for (int i = j + tid; i < n; i += NT) W(3, i, j) = (i == j) ? 1.0 : W(4, i, j) * scl;
      __syncthreads();
      if (tau != 0.0) {
        for (int c = j + 1 + tid; c < h; c += NT) {  // one thread per column
          double dot = 0.0;
          for (int i = j; i < n; ++i) dot += W(3, i, j) * W(4, i, c);
          dot *= tau;
          for (int i = j; i < n; ++i) W(4, i, c) -= dot * W(3, i, j);
        }
      }
      __syncthreads();
    }
    for (int c = h + tid; c < nvec; c += NT) {
      for (int i = 0; i < n; ++i) Z(i, c) = (i == c) ? 1.0 : 0.0;
      for (int j = h - 1; j >= 0; --j) {
        const double tau = rtau[j];
        if (tau == 0.0) continue;
        double dot = 0.0;
        for (int i = j; i < n; ++i) dot += W(3, i, j) * Z(i, c);
        dot *= tau;
        for (int i = j; i < n; ++i) Z(i, c) -= dot * W(3, i, j);
      }
    }
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
