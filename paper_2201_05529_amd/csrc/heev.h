// Batched Hermitian eigensolver in double precision, one workgroup per
// problem.  Used for every Gram matrix of the bond update (the truncated
// SVDs of Appendix A.2 are computed from Gram matrices).
//
//  stage 1  (its own kernel) Householder reduction A = Q T Q^H, T real
//           symmetric tridiagonal (reflector H_j = I - tau_j v_j v_j^H,
//           H_j^H x = beta e_1)
//  stage 2  off-diagonal entries of T at the rounding level of |T| are set
//           to zero, which splits T into unreduced blocks; then
//           T + delta I = L D L^T with D > 0 (delta a few ulps of |T|, more
//           if needed, so the factorisation exists)
//  stage 3  every eigenvalue of each block of L D L^T: a shared grid of qd
//           negative counts brackets all of them, then multisection to high
//           relative accuracy; the values of all blocks are merged into one
//           descending list that remembers each value's block; then the
//           selection rule (truncated-SVD rule of Appendix A.2, or a
//           numerical-rank rule) fixes how many leading eigenpairs are
//           needed
//  stage 4  their eigenvectors of T from twisted factorisations of their
//           own block (one O(block) solve per vector, zero outside the
//           block); within a block, clusters of numerically equal eigenvalues
//           get random starts, inverse iteration and Gram-Schmidt against
//           the cluster and its near neighbours; eigenvalues within the
//           rounding level of zero (the numerical null space of a singular
//           Gram matrix) form one cluster over all blocks, orthogonalised
//           against all other vectors.  Equal eigenvalues of different
//           blocks (exact degeneracies, common in Gram matrices of
//           symmetric states) need no special care: their vectors have
//           disjoint supports
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
  int* status;       // sticky error word (bit 1: no convergence, bit 4: non-finite, bit 8: size above n_cap);
                     // the bond update folds it into the stepped chain's status
  int noise_cluster; // 1: eigenvalues at the rounding level of zero form one cluster (stage 4b)
  const double* abs_ref;  // RULE_RANK: if set, also drop eigenvalues <= abs_tol * (*abs_ref),
  double abs_tol;         //            and allow no eigenpair at all
  unsigned long long* stamps;  // if set: wall-clock stamps at the stage boundaries [8] (profiling)
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
  // unrolled so that the reads of d and lld, which do not depend on the
  // recurrence, are issued ahead of it
#pragma unroll 4
  for (int i = 0; i + 1 < n; ++i) {
    double dp = d[i] + s;
    if (fabs(dp) < pivmin) dp = -pivmin;
    cnt += dp < 0.0;
    // 1 / dp from the hardware estimate and two Newton steps (a rounding-
    // level relative perturbation of each step, which the count tolerates
    // as the factorisation's own rounding), cheaper than a full division
    double r = __builtin_amdgcn_rcp(dp);
    double e = fma(-dp, r, 1.0);
    r = fma(r, e, r);
    e = fma(-dp, r, 1.0);
    r = fma(r, e, r);
    s = lld[i] * (s * r) - sigma;
  }
  double dp = d[n - 1] + s;
  if (fabs(dp) < pivmin) dp = -pivmin;
  cnt += dp < 0.0;
  return cnt;
}

// ------------------------------------------------------------- stage 1
// Reduction to real tridiagonal form, T = Q^H A Q (its own kernel, one
// workgroup per problem; writes d, e, tau and the reflectors).
//
// Both triangles of the trailing block are kept.  The rank-2 update of step
// j is not applied at once: step j+1 first forms its own row from the
// pending update, then one fused pass over the trailing block applies the
// pending update and accumulates the next matrix-vector product, so every
// element is visited once per step.  Each element needs three entries of
// the step's vectors (w_r, v_r of the pending update and the new reflector
// v_r) that are the same for the whole row; a thread owns two columns, so
// each such LDS read serves two elements.  While the trailing
// block is larger than TRI_RES the pass reads and writes it in global
// memory, coalesced along rows (lane p owns columns p and p + ceil(m/2)),
// with the loads of the next batch of TRI_DEPTH rows issued while the
// current batch is updated.  Once it fits, the block moves into registers (wave w holds rows
// w + 8 k, lane l columns 2 l and 2 l + 1: 128 registers per thread, which
// eight waves of 256 registers hold without spilling) and the remaining
// steps touch no memory but the vectors in LDS; the row that the next step
// reflects is handed over through LDS.
constexpr int HEEV_TRI_THREADS = 512;
constexpr int TRI_RES = 128;
constexpr int TRI_WAVES = HEEV_TRI_THREADS / 64;
constexpr int TRI_RES_ROWS = TRI_RES / TRI_WAVES;
constexpr int TRI_DEPTH = 4;

// flops (may be null): accumulates the algorithmic flop count of the
// reduction, 16 n^3 / 3 per complex Hermitian matrix.
__global__ void __launch_bounds__(HEEV_TRI_THREADS) heev_tridiag_kernel(const HeevJob* jobs, double* flops) {
  constexpr int NT = HEEV_TRI_THREADS;
  const HeevJob& J = jobs[blockIdx.x];
  const int n = *J.n_ptr;
  const int tid = threadIdx.x;
  if (n > J.n_cap || n <= 0) return;  // the solve kernel reports a size beyond the workspace
  if (flops && tid == 0) atomicAdd(flops, 16.0 / 3.0 * (double)n * n * n);
  if (J.stamps && tid == 0) J.stamps[0] = wall_clock64();
  __shared__ double2 vbuf[2][1024];
  __shared__ double2 sy[1024];      // tau A v of the pending step (w = y - half v)
  __shared__ double2 part[1024];    // partial matrix-vector sums [groups][m]
  __shared__ double2 rowbuf[TRI_RES];
  __shared__ double s_dd[1024], s_ee[1024];   // T, written out at the end
  __shared__ double2 s_tau[1024];
  __shared__ double s_sig[TRI_WAVES];    // |x|^2 below the first entry, per wave
  __shared__ double2 s_vhy[TRI_WAVES];   // v^H y, per wave
  __shared__ double2 s_alpha;
  double2* A = J.a;
  const int lda = J.lda;
  const int nc = J.n_cap;
  // the wave index, known to the compiler as uniform across the wave
  const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  double2* vp = vbuf[0];          // pending v (offset j at step j)
  double2* vc = vbuf[1];          // current v
  double half = 0.0;              // of the pending step
  // before the first step the pending update is zero (w = 0, v = 0)
  for (int i = tid; i < 1024; i += NT) {
    vp[i] = mk<double>(0.0, 0.0);
    sy[i] = mk<double>(0.0, 0.0);
  }
  __syncthreads();

  // w_i of the pending update, w = y - half v
  auto wpend = [&](int i) { return csub<double>(sy[i], cscale<double>(vp[i], half)); };
  // val -= w_r conj(v_c) + v_r conj(w_c), as eight fused multiply-adds
  auto update = [&](double2& val, double2 wr, double2 vr, double2 wc, double2 vcol) {
    val.x = fma(-wr.x, vcol.x, val.x);
    val.x = fma(-wr.y, vcol.y, val.x);
    val.x = fma(-vr.x, wc.x, val.x);
    val.x = fma(-vr.y, wc.y, val.x);
    val.y = fma(-wr.y, vcol.x, val.y);
    val.y = fma(wr.x, vcol.y, val.y);
    val.y = fma(-vr.y, wc.x, val.y);
    val.y = fma(vr.x, wc.y, val.y);
  };

  // (a) row j of the updated matrix (row(i) = A_j,j+1+i, row(-1) the
  // diagonal, before the pending update); x = conj(row) below the diagonal;
  // (b) the reflector, computed redundantly by every thread, into vc.
  // Per-wave partial sums are added in a fixed order (bit-reproducible):
  // lane q takes wave q's, then a DPP sum over the wave.
  auto reflect = [&](int j, auto row) {
    const int m = n - j - 1;
    double p2 = 0.0;
    for (int i = tid; i < m; i += NT) {
      double2 val = row(i);
      update(val, wpend(0), vp[0], wpend(i + 1), vp[i + 1]);
      const double2 x = cconj<double>(val);
      vc[i] = x;
      if (i == 0) s_alpha = x;
      else p2 += cabs2<double>(x);
    }
    p2 = wave_sum_dpp(p2);
    if (lane == 0) s_sig[wid] = p2;
    if (tid == 0) {
      const double2 w0 = wpend(0);
      s_dd[j] = row(-1).x - 2.0 * (w0.x * vp[0].x + w0.y * vp[0].y);
    }
    __syncthreads();
    const double sig2 = wave_sum_dpp(lane < TRI_WAVES ? s_sig[lane] : 0.0);
    const double2 alpha = s_alpha;
    double2 tau = mk<double>(0.0, 0.0);
    double beta = alpha.x;
    if (!(sig2 == 0.0 && alpha.y == 0.0)) {
      const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig2);
      beta = alpha.x >= 0.0 ? -nrm : nrm;
      const double ib = 1.0 / beta;
      tau = mk<double>((beta - alpha.x) * ib, -alpha.y * ib);
    }
    const bool active = !(tau.x == 0.0 && tau.y == 0.0);
    double2 scal = mk<double>(0.0, 0.0);
    {
      const double2 den = mk<double>(alpha.x - beta, alpha.y);
      const double dn = den.x * den.x + den.y * den.y;
      if (active && dn > 0.0) {
        const double idn = 1.0 / dn;
        scal = mk<double>(den.x * idn, -den.y * idn);
      }
    }
    if (tid == 0) {
      s_tau[j] = tau;
      s_ee[j] = beta;
    }
    for (int i = tid; i < m; i += NT) {
      const double2 vi = (i == 0) ? mk<double>(1.0, 0.0)
                                  : (active ? cmul<double>(vc[i], scal) : mk<double>(0.0, 0.0));
      vc[i] = vi;
      gstore(J.refl + (size_t)j * nc + i, vi);
    }
    __syncthreads();
    return tau;
  };

  // (d) y = tau A22 v from the partial sums (kept in sy), v^H y; the
  // update w = y - 1/2 Re(conj(tau) v^H y) v becomes the pending one
  auto finish = [&](int m, int groups, double2 tau) {
    double2 pv = mk<double>(0.0, 0.0);
    for (int i = tid; i < m; i += NT) {
      double2 y = mk<double>(0.0, 0.0);
      for (int q = 0; q < groups; ++q) y = cadd<double>(y, part[q * m + i]);
      y = cmul<double>(tau, y);
      sy[i] = y;
      cfmaconj<double>(pv, vc[i], y);
    }
    pv.x = wave_sum_dpp(pv.x);
    pv.y = wave_sum_dpp(pv.y);
    if (lane == 0) s_vhy[wid] = pv;
    __syncthreads();
    const double2 q = lane < TRI_WAVES ? s_vhy[lane] : mk<double>(0.0, 0.0);
    const double2 vhy = mk<double>(wave_sum_dpp(q.x), wave_sum_dpp(q.y));
    half = 0.5 * (tau.x * vhy.x + tau.y * vhy.y);
    double2* t = vp;
    vp = vc;
    vc = t;
  };

  // steps with a trailing block larger than TRI_RES: global memory
  const int j0 = max(0, n - TRI_RES);
  for (int j = 0; j < j0; ++j) {
    const int m = n - j - 1, off = j + 1;
    const double2* arow = A + (size_t)j * lda + off;
    const double2 tau = reflect(j, [&](int i) { return gload(arow + i); });
    // (c) fused pass: A22 -= pending update; part = conj(A22)^T v.  Thread
    // (g, p) owns columns p and p + mp of A22 (the second one only if m is
    // larger), so each load and store instruction covers contiguous
    // columns, and rows g, g + groups, ...
    const int mp = (m + 1) >> 1;
    const int groups = max(1, NT / mp);
    const int p = tid % mp, g = tid / mp;
    if (g < groups) {
      const int c0 = p, c1 = min(p + mp, m - 1);
      const bool two = p + mp < m;
      double2 acc0 = mk<double>(0.0, 0.0), acc1 = mk<double>(0.0, 0.0);
      double2* base = A + (size_t)off * lda + off;
      const double2 wc0 = wpend(c0 + 1), vc0 = vp[c0 + 1], wc1 = wpend(c1 + 1), vc1 = vp[c1 + 1];
      // two batches of TRI_DEPTH rows in flight: the next batch is loaded
      // while the current one is updated.  Loads of rows past the end
      // re-read the last row (no branch around a load); only the rows
      // inside are updated and summed
      const int stride = TRI_DEPTH * groups;
      auto load_batch = [&](int r0, double2* x0, double2* x1) {
#pragma unroll
        for (int u = 0; u < TRI_DEPTH; ++u) {
          const int r = min(r0 + u * groups, m - 1);
          x0[u] = gload(base + r * lda + c0);
          x1[u] = gload(base + r * lda + c1);
        }
      };
      auto run_batch = [&](int r0, double2* x0, double2* x1) {
#pragma unroll
        for (int u = 0; u < TRI_DEPTH; ++u) {
          const int r = r0 + u * groups;
          if (r < m) {
            const double2 vr = vc[r];
            const double2 wr = wpend(r + 1), pr = vp[r + 1];
            update(x0[u], wr, pr, wc0, vc0);
            update(x1[u], wr, pr, wc1, vc1);
            gstore(base + r * lda + c0, x0[u]);
            if (two) gstore(base + r * lda + c1, x1[u]);
            cfmaconj<double>(acc0, x0[u], vr);
            cfmaconj<double>(acc1, x1[u], vr);
          }
        }
      };
      double2 a0[TRI_DEPTH], a1[TRI_DEPTH], b0[TRI_DEPTH], b1[TRI_DEPTH];
      int r0 = g;
      load_batch(r0, a0, a1);
      while (r0 < m) {
        load_batch(r0 + stride, b0, b1);
        run_batch(r0, a0, a1);
        r0 += stride;
        if (r0 >= m) break;
        load_batch(r0 + stride, a0, a1);
        run_batch(r0, b0, b1);
        r0 += stride;
      }
      part[g * m + c0] = acc0;
      if (two) part[g * m + c1] = acc1;
    }
    __syncthreads();
    finish(m, groups, tau);
  }

  // the trailing block [j0, n)^2 (updated up to the pending step) into
  // registers: ar[k][h] = A_(j0 + wid + 8 k),(j0 + 2 lane + h)
  const int nr = n - j0;
  double2 ar[TRI_RES_ROWS][2];
#pragma unroll
  for (int k = 0; k < TRI_RES_ROWS; ++k) {
    const int r = wid + TRI_WAVES * k;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 2 * lane + h;
      ar[k][h] = (r < nr && c < nr) ? gload(A + (size_t)(j0 + r) * lda + j0 + c) : mk<double>(0.0, 0.0);
    }
  }
  if (wid == 0) {
    if (2 * lane < nr) rowbuf[2 * lane] = ar[0][0];
    if (2 * lane + 1 < nr) rowbuf[2 * lane + 1] = ar[0][1];
  }
  __syncthreads();
  for (int j = j0; j + 1 < n; ++j) {
    const int m = n - j - 1, ol = j + 1 - j0;   // ol: first row / column of A22 in the block
    const double2 tau = reflect(j, [&](int i) { return rowbuf[ol + i]; });
    // (c) on the registers: lane columns 2 lane + h are A22 columns
    // cc_h = 2 lane + h - ol; the first row of A22 goes to rowbuf
    const int cc0 = 2 * lane - ol, cc1 = cc0 + 1;
    const bool ok0 = cc0 >= 0 && cc0 < m, ok1 = cc1 >= 0 && cc1 < m;
    if (ok0 || ok1) {
      double2 acc0 = mk<double>(0.0, 0.0), acc1 = mk<double>(0.0, 0.0);
      // a column outside A22 reads index 0 and is never stored
      const int i0 = ok0 ? cc0 + 1 : 0, i1 = ok1 ? cc1 + 1 : 0;
      const double2 wc0 = wpend(i0), vc0 = vp[i0], wc1 = wpend(i1), vc1 = vp[i1];
#pragma unroll
      for (int k = 0; k < TRI_RES_ROWS; ++k) {
        const int rr = wid + TRI_WAVES * k - ol;   // row of A22, the same for the whole wave
        if (rr >= 0 && rr < m) {
          const double2 vr = vc[rr];
          const double2 wr = wpend(rr + 1), pr = vp[rr + 1];
          update(ar[k][0], wr, pr, wc0, vc0);
          update(ar[k][1], wr, pr, wc1, vc1);
          if (rr == 0) {
            if (ok0) rowbuf[ol + cc0] = ar[k][0];
            if (ok1) rowbuf[ol + cc1] = ar[k][1];
          }
          cfmaconj<double>(acc0, ar[k][0], vr);
          cfmaconj<double>(acc1, ar[k][1], vr);
        }
      }
      if (ok0) part[wid * m + cc0] = acc0;
      if (ok1) part[wid * m + cc1] = acc1;
    }
    __syncthreads();
    finish(m, TRI_WAVES, tau);
  }
  if (tid == 0) {
    const double2 w0 = wpend(0);
    s_dd[n - 1] = (n > 1 ? rowbuf[nr - 1].x : gload(A).x) - 2.0 * (w0.x * vp[0].x + w0.y * vp[0].y);
    s_ee[n - 1] = 0.0;
    s_tau[n - 1] = mk<double>(0.0, 0.0);
  }
  __syncthreads();
  // T and the reflector scalars: d, e, tau (re, im)
  for (int i = tid; i < n; i += NT) {
    gstore(J.tri + i, s_dd[i]);
    gstore(J.tri + nc + i, s_ee[i]);
    gstore(reinterpret_cast<double2*>(J.tri + 2 * nc) + i, s_tau[i]);
  }
  if (J.stamps && tid == 0) J.stamps[1] = wall_clock64();
}

// ------------------------------------------------------------- stage 2..4
// After heev_tridiag_kernel on the same jobs: d, e of T are in J.tri.
__global__ void __launch_bounds__(HEEV_SOLVE_THREADS) heev_solve_kernel(const HeevJob* jobs) {
  constexpr int NT = HEEV_SOLVE_THREADS;
  const HeevJob& J = jobs[blockIdx.x];
  const int n = *J.n_ptr;
  const int tid = threadIdx.x;
  if (n > J.n_cap) {  // a size beyond the workspace: refuse (status bit 8)
    if (tid == 0) atomicOr(J.status, 8);
    return;
  }
  if (n <= 0) return;  // nothing to do; *nvec_out is left as it is
  auto stamp = [&](int i) {
    if (J.stamps && tid == 0) J.stamps[i] = wall_clock64();
  };
  __shared__ double buf[8192];     // d, l, l d, l^2 d, mu, tau, inverse-iteration scratch
  __shared__ double red[NT / 64];
  __shared__ double2 s_tau;
  __shared__ double s_beta, s_delta, s_tnorm;
  __shared__ int s_nvec, s_ok, s_nb, s_nref;
  __shared__ int s_bs[1025];  // block b of T covers rows [s_bs[b], s_bs[b + 1])
  __shared__ int s_kb[1024];  // block of the eigenvalue mu[j] (ascending order)
  const int nc = J.n_cap;
  double* dd = J.tri;              // diagonal of T
  double* ee = J.tri + nc;         // off-diagonal of T (ee[i] couples i, i+1)

  // -------- stage 2: T + delta I = L D L^T with D > 0
  double* d = buf;
  double* l = buf + 1024;
  double* ld = buf + 2048;
  double* lld = buf + 3072;
  double* mu = buf + 4096;
  // T staged in LDS for the sequential loops of thread 0 (the slots are
  // stage 3's, written only after this stage)
  double* sdd = buf + 5120;
  double* see = buf + 6144;
  for (int i = tid; i < n; i += NT) {
    sdd[i] = gload(dd + i);
    see[i] = gload(ee + i);
  }
  __syncthreads();
  if (tid == 0) {
    double tn = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = fabs(sdd[i]) + (i > 0 ? fabs(see[i - 1]) : 0.0) + (i + 1 < n ? fabs(see[i]) : 0.0);
      tn = fmax(tn, r);
    }
    s_tnorm = tn;
    // split T where a coupling is at the rounding level of |T| (a
    // perturbation of T no larger than the rounding errors of stage 1)
    int nb = 0;
    s_bs[0] = 0;
    for (int i = 0; i + 1 < n; ++i)
      if (fabs(see[i]) <= 2.2e-16 * tn) {
        see[i] = 0.0;
        gstore(ee + i, 0.0);
        s_bs[++nb] = i + 1;
      }
    s_bs[++nb] = n;
    s_nb = nb;
    int ok = 0;
    double delta = fmax(8.0 * n * 2.2e-16 * tn, 1e-300);
    if (tn > 0.0) {
      for (int attempt = 0; attempt < 64 && !ok; ++attempt) {
        ok = 1;
        double di = sdd[0] + delta;
        for (int i = 0; i < n; ++i) {
          if (!(di > 1e-300 * fmax(tn, 1.0))) { ok = 0; break; }
          d[i] = di;
          if (i + 1 < n) {
            const double li = see[i] / di;
            l[i] = li;
            ld[i] = li * di;
            lld[i] = li * li * di;
            di = (sdd[i + 1] + delta) - li * see[i];
          }
        }
        if (!ok) delta = fmin(delta * 8.0, 4.0 * tn);
      }
    }
    s_delta = delta;
    s_ok = ok;
  }
  __syncthreads();
  stamp(2);
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
    // -------- stage 3: eigenvalues of each block of L D L^T (the qd
    // recurrence restarts at a split, so a count over the whole matrix is
    // the sum of the blocks' counts).  (a) one shared pass: every thread
    // counts the eigenvalues below one point of a geometric grid over
    // [1e-40 top, top], which brackets every eigenvalue to a factor 1.1;
    // (b) each is refined by multisection with a group of te threads
    // (te + 1 geometric subintervals per round) down to a few ulps
    // (relative accuracy).  Slot g holds eigenvalue g - s_bs[b] (ascending)
    // of the block b that contains row g.
    const double pivmin = 1e-290 * fmax(1.0, tnorm * tnorm);
    const int nb = s_nb;
    double* xg = buf + 6144;
    int* cg = reinterpret_cast<int*>(buf + 7168);
    double* val = (nb > 1) ? buf + 5120 : mu;  // slot values (merged into mu below)
    const double top = 1.01 * (tnorm + delta) + 1e-300;
    const double bot = fmax(1e-40 * top, 1e-300);
    {
      const double x = bot * exp((double)tid / (NT - 1) * log(top / bot));
      xg[tid] = x;
      cg[tid] = (nb == 1) ? ldl_negcount(d, lld, n, x, pivmin) : 0;
    }
    __syncthreads();
    int te = 1;
    while (te < 64 && te * 2 * max(n, 1) <= NT) te *= 2;
    const int q = tid % te;
    const int base = (tid & 63) & ~(te - 1);
    for (int g0 = 0; g0 < n; g0 += NT / te) {
      const int g = g0 + tid / te;
      double lo = 0.0, hi = 0.0;
      if (g < n) {
        int b = 0;
        if (nb > 1) {  // last block starting at or before row g
          int a = 0, c = nb;
          while (c - a > 1) {
            const int m = (a + c) >> 1;
            if (s_bs[m] <= g) a = m;
            else c = m;
          }
          b = a;
        }
        const int r0 = s_bs[b], len = s_bs[b + 1] - r0, k = g - r0;
        const double* db = d + r0;
        const double* lb = lld + r0;
        // first grid point with more than k eigenvalues of the block below
        int a = 0, c = NT;
        while (a < c) {
          const int m = (a + c) >> 1;
          const int cnt = (nb == 1) ? cg[m] : ldl_negcount(db, lb, len, xg[m], pivmin);
          if (cnt > k) c = m;
          else a = m + 1;
        }
        hi = (a < NT) ? xg[a] : top;
        lo = (a > 0) ? xg[a - 1] : 1e-300 * top;
        const double f = (q + 1) / (double)(te + 1);
        for (int it = 0; it < 120; ++it) {
          if (hi - lo <= 4.4e-16 * hi) break;
          const bool geo = lo > 0.0 && hi > 4.0 * lo;
          const double x = geo ? lo * exp(f * log(hi / lo)) : lo + f * (hi - lo);
          const int cnt = ldl_negcount(db, lb, len, x, pivmin);
          double nlo = lo, nhi = hi;
          for (int r = 0; r < te; ++r) {
            const double xr = __shfl(x, base + r, 64);
            const int cr = __shfl(cnt, base + r, 64);
            if (cr <= k) nlo = fmax(nlo, xr);
            else nhi = fmin(nhi, xr);
          }
          lo = nlo;
          hi = nhi;
        }
        if (q == 0) {
          val[g] = 0.5 * (lo + hi);
          if (nb == 1) s_kb[g] = 0;
        }
      }
    }
    __syncthreads();
    if (nb > 1) {
      // merge: ascending position of slot g = number of smaller values
      // (equal values ordered by slot)
      for (int g = tid; g < n; g += NT) {
        const double v = val[g];
        int pos = 0;
        for (int h = 0; h < n; ++h) {
          const double u = val[h];
          pos += (u < v) || (u == v && h < g);
        }
        int a = 0, c = nb;
        while (c - a > 1) {
          const int m = (a + c) >> 1;
          if (s_bs[m] <= g) a = m;
          else c = m;
        }
        mu[pos] = v;
        s_kb[pos] = a;
      }
      __syncthreads();
    }
    for (int j = tid; j < n; j += NT) J.w[n - 1 - j] = mu[j] - delta;
  }
  __syncthreads();
  stamp(3);

  // -------- stage 3b: selection rule (thread 0)
  if (tid == 0) {
    const double* w = J.w;
    int nvec = 0;
    const double lam0 = w[0];
    if (J.rule == RULE_FULL) {
      nvec = n;
    } else if (J.rule == RULE_RANK) {
      const double floor_abs = J.abs_ref ? J.abs_tol * fmax(*J.abs_ref, 0.0) : 0.0;
      while (nvec < n && w[nvec] > J.rank_tol * lam0 && w[nvec] > floor_abs && w[nvec] > 0.0) ++nvec;
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
        // runs of singular values within a relative gap of 1e-6 are kept
        // or dropped whole: an eps cut inside one moves to its end, a cap
        // inside one to its start
        auto in_run = [&](int k) {
          const double a = sqrt(fmax(w[k - 1], 0.0)), b = sqrt(fmax(w[k], 0.0));
          return a - b < 1e-6 * a;
        };
        while (nvec < npos && in_run(nvec)) ++nvec;
        if (J.rule == RULE_CAP && J.cap > 0 && nvec > J.cap) {
          nvec = J.cap;
          while (nvec > 1 && in_run(nvec)) --nvec;
        }
      }
    }
    if (nvec < 1 && lam0 > 0.0 && !(J.rule == RULE_RANK && J.abs_ref)) nvec = 1;
    if (!(lam0 == lam0) || isinf(lam0)) atomicOr(J.status, 4);
    s_nvec = nvec;
    *J.nvec_out = nvec;
  }
  __syncthreads();
  stamp(4);
  const int nvec = s_nvec;

  // -------- stage 4: eigenvectors of T by twisted factorisations of
  // L D L^T - mu I (one thread per vector), the method of Dhillon and
  // Parlett (Linear Algebra Appl. 387, 2004; the vectors of MRRR without its
  // representation tree: clusters are handled in stage 4b).  Top-down: D+_i = d_i + s_i,
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
  const int nres = nvec;
  // rows [r0, r1) of the block that holds the eigenvalue of descending index k
  auto block_of = [&](int k, int& r0, int& r1) {
    const int b = s_kb[n - 1 - k];
    r0 = s_bs[b];
    r1 = s_bs[b + 1];
  };
  // x / y from the hardware reciprocal and two Newton steps (a rounding-level
  // perturbation, which the factorisations tolerate as their own rounding)
  auto qdiv = [](double x, double y) {
    double r = __builtin_amdgcn_rcp(y);
    double e = fma(-y, r, 1.0);
    r = fma(r, e, r);
    e = fma(-y, r, 1.0);
    r = fma(r, e, r);
    return x * r;
  };
  // the per-vector arrays in global memory, through global-space accesses;
  // the loops that read back what they stored load TWIST_AHEAD entries ahead
  constexpr int TWIST_AHEAD = 4;
  auto wld = [&](int arr, int i, int k) { return gload(&J.work[((size_t)arr * nc + i) * nc + k]); };
  auto wst = [&](int arr, int i, int k, double v) { gstore(&J.work[((size_t)arr * nc + i) * nc + k], v); };
  auto zst = [&](int i, int k, double v) { gstore(&J.z[(size_t)i * nc + k], v); };
  auto zld = [&](int i, int k) { return gload(&J.z[(size_t)i * nc + k]); };
  for (int k = tid; k < nres; k += NT) {
    const double m_k = mu[n - 1 - k];
    int r0, r1;
    block_of(k, r0, r1);
    // top-down (stationary)
    double s = -m_k;
    for (int i = r0; i + 1 < r1; ++i) {
      wst(1, i, k, s);
      double dp = d[i] + s;
      if (fabs(dp) < pivmin) dp = dp < 0.0 ? -pivmin : pivmin;
      const double idp = qdiv(1.0, dp);
      wst(0, i, k, ld[i] * idp);
      s = lld[i] * (s * idp) - m_k;
    }
    wst(1, r1 - 1, k, s);
    // bottom-up (progressive) with the twist index
    double p = d[r1 - 1] - m_k;
    double gmin = fabs(s + p + m_k);
    int r = r1 - 1;
    for (int i0 = r1 - 2; i0 >= r0; i0 -= TWIST_AHEAD) {
      double sv[TWIST_AHEAD];
#pragma unroll
      for (int u = 0; u < TWIST_AHEAD; ++u) sv[u] = wld(1, max(i0 - u, r0), k);
#pragma unroll
      for (int u = 0; u < TWIST_AHEAD; ++u) {
        const int i = i0 - u;
        if (i >= r0) {
          double dm = lld[i] + p;
          if (fabs(dm) < pivmin) dm = dm < 0.0 ? -pivmin : pivmin;
          const double t = qdiv(d[i], dm);
          wst(2, i, k, l[i] * t);
          p = p * t - m_k;
          const double g = fabs(sv[u] + p + m_k);
          if (g < gmin) { gmin = g; r = i; }
        }
      }
    }
    // solve
    double z = 1.0, nrm = 1.0;
    zst(r, k, 1.0);
    for (int i0 = r - 1; i0 >= r0; i0 -= TWIST_AHEAD) {
      double wv[TWIST_AHEAD];
#pragma unroll
      for (int u = 0; u < TWIST_AHEAD; ++u) wv[u] = wld(0, max(i0 - u, r0), k);
#pragma unroll
      for (int u = 0; u < TWIST_AHEAD; ++u) {
        const int i = i0 - u;
        if (i >= r0) {
          z = -wv[u] * z;
          zst(i, k, z);
          nrm += z * z;
        }
      }
    }
    z = 1.0;
    for (int i0 = r; i0 + 1 < r1; i0 += TWIST_AHEAD) {
      double wv[TWIST_AHEAD];
#pragma unroll
      for (int u = 0; u < TWIST_AHEAD; ++u) wv[u] = wld(2, min(i0 + u, r1 - 2), k);
#pragma unroll
      for (int u = 0; u < TWIST_AHEAD; ++u) {
        const int i = i0 + u;
        if (i + 1 < r1) {
          z = -wv[u] * z;
          zst(i + 1, k, z);
          nrm += z * z;
        }
      }
    }
    const double inv = (nrm > 0.0 && nrm < 1e300) ? 1.0 / sqrt(nrm) : 0.0;
    for (int i = 0; i < n; ++i) {
      const bool in = i >= r0 && i < r1;
      // overflow: fall back to the unit vector at the twist index
      zst(i, k, !in ? 0.0 : (inv > 0.0 ? zld(i, k) * inv : (i == r ? 1.0 : 0.0)));
    }
  }
  __syncthreads();
  stamp(5);

  // -------- stage 4b: clusters of numerically equal eigenvalues (relative
  // gap below 1e-9) inside one block.  Twisted vectors of equal mu
  // coincide, so every member after the first restarts from a seeded random
  // vector on the block's rows and takes three inverse-iteration solves
  // (pivoted elimination of the block of T - lambda I); after each solve it
  // is orthogonalised against the vectors of its block near it that are
  // already final (the twisted ones and the earlier members of its cluster),
  // since the solve alone amplifies whichever member of the cluster has the
  // smallest pivot and would lose the others to rounding.  Members of
  // different clusters run in parallel, the r-th members of all clusters in
  // round r.  Clusters of more than four values (near-multiples of the
  // identity on a block) skip the per-solve projection and take all their
  // members in the first round: their solves amplify the members evenly.  A
  // final Gram-Schmidt over the members in order follows.  Eigenvalues of T within delta of zero are rounding noise of a
  // (numerically) singular matrix, not values known to any relative
  // accuracy: they form one cluster over all blocks whatever their relative
  // gaps, every member of it (the first one too) is a seeded random vector
  // of the whole space, and each is orthogonalised against all other
  // vectors.
  {
    const double rgap = 1e-9;
    // |lambda| below the initial shift (8 n eps |T|) is rounding noise;
    // mu = lambda + delta
    const double noise = 8.0 * n * 2.2e-16 * tnorm;
    const bool use_noise = J.noise_cluster != 0;
    auto is_noise = [&](int a) { return use_noise && fabs(mu[n - 1 - a] - delta) <= noise; };
    auto close = [&](int a, int b) {  // a, b descending-order indices
      const double ma = mu[n - 1 - a], mb = mu[n - 1 - b];
      return fabs(ma - mb) <= rgap * fmax(fabs(ma), fabs(mb));
    };
    // k repeats the eigenvalue of an earlier index of its own block (the
    // indices between two close values hold close values too)
    // number of earlier indices of k's block with a close eigenvalue (0: not
    // a member)
    auto member_rank = [&](int k) {
      if (is_noise(k)) return 0;
      const int bk = s_kb[n - 1 - k];
      int r = 0;
      for (int i = k - 1; i >= 0 && close(i, k); --i) r += s_kb[n - 1 - i] == bk;
      return r;
    };
    auto is_member = [&](int k) { return member_rank(k) > 0; };
    constexpr int SMALL_CLUSTER = 4;
    // more than SMALL_CLUSTER same-block values close to k's
    auto big_cluster = [&](int k) {
      if (is_noise(k)) return false;
      const int bk = s_kb[n - 1 - k];
      int c = 1;
      for (int i = k - 1; i >= 0 && close(i, k) && c <= SMALL_CLUSTER; --i) c += s_kb[n - 1 - i] == bk;
      for (int i = k + 1; i < nres && close(i, k) && c <= SMALL_CLUSTER; ++i) c += s_kb[n - 1 - i] == bk;
      return c > SMALL_CLUSTER;
    };
    auto near = [&](int a, int b) {
      const double ma = mu[n - 1 - a], mb = mu[n - 1 - b];
      return fabs(ma - mb) <= 1e-3 * fmax(fabs(ma), fabs(mb));
    };
    // pivots of the (nearly) singular shifted matrix are floored at
    // eps |T|, as in inverse iteration: the solve then amplifies the
    // eigenspace without overflowing
    const double pfloor = fmax(2.2e-16 * tnorm, pivmin);
    for (int k = tid; k < nres; k += NT)
      if (is_noise(k)) {
        // any vector of the null space will do: a seeded random start,
        // projected onto the complement of the other vectors below
        for (int i = 0; i < n; ++i) Z(i, k) = u01(splitmix64(0xA24BAED4963EE407ull * (k + 1) + i)) - 0.5;
      }
    for (int round = 1; round < SMALL_CLUSTER; ++round) {
      for (int k = tid; k < nres; k += NT) {
        const int rk = member_rank(k);
        const bool big = rk > 0 && big_cluster(k);
        if (big ? round != 1 : rk != round) continue;
        // inverse iteration on the rows [r0, r1) of the block, T - lambda I
        // factored by Gaussian elimination with partial pivoting (bounded
        // growth; pivots floored at eps |T|)
        int r0, r1;
        block_of(k, r0, r1);
        const int bk = s_kb[n - 1 - k];
        int na = k, nb = k + 1;
        while (na > 0 && near(na - 1, k)) --na;
        while (nb < nres && near(nb, k)) ++nb;
        // final vectors of the block near k: twisted ones and members of
        // small clusters from earlier rounds
        auto final_ref = [&](int i) {
          if (i == k || s_kb[n - 1 - i] != bk || is_noise(i)) return false;
          const int ri = member_rank(i);
          return ri == 0 || (ri < round && !big_cluster(i));
        };
        const double lam = mu[n - 1 - k] - delta;
        for (int i = r0; i < r1; ++i) {
          W(0, i, k) = (i + 1 < r1) ? ee[i] : 0.0;  // sub-diagonal, then multipliers
          W(1, i, k) = dd[i] - lam;                 // diagonal of U
          W(2, i, k) = (i + 1 < r1) ? ee[i] : 0.0;  // first super-diagonal of U
          W(3, i, k) = 0.0;                         // second super-diagonal of U
          W(4, i, k) = 0.0;                         // row swap at step i
        }
        for (int i = r0; i + 1 < r1; ++i) {
          const double di = W(1, i, k), li = W(0, i, k);
          if (fabs(di) >= fabs(li)) {
            W(0, i, k) = (di != 0.0) ? li / di : 0.0;
            W(1, i + 1, k) -= W(0, i, k) * W(2, i, k);
          } else {
            const double f = di / li;
            W(1, i, k) = li;
            W(0, i, k) = f;
            const double tmp = W(2, i, k);
            W(2, i, k) = W(1, i + 1, k);
            W(1, i + 1, k) = tmp - f * W(1, i + 1, k);
            if (i + 2 < r1) {
              W(3, i, k) = W(2, i + 1, k);
              W(2, i + 1, k) = -f * W(2, i + 1, k);
            }
            W(4, i, k) = 1.0;
          }
        }
        for (int i = r0; i < r1; ++i)
          if (fabs(W(1, i, k)) < pfloor) W(1, i, k) = W(1, i, k) >= 0.0 ? pfloor : -pfloor;
        for (int i = r0; i < r1; ++i) W(5, i, k) = u01(splitmix64(0xA24BAED4963EE407ull * (k + 1) + i)) - 0.5;
        for (int it = 0; it < 3; ++it) {
          for (int i = r0; i + 1 < r1; ++i) {  // P, L
            if (W(4, i, k) != 0.0) {
              const double t = W(5, i, k);
              W(5, i, k) = W(5, i + 1, k);
              W(5, i + 1, k) = t;
            }
            W(5, i + 1, k) -= W(0, i, k) * W(5, i, k);
          }
          for (int i = r1 - 1; i >= r0; --i) {  // U
            double acc = W(5, i, k);
            if (i + 1 < r1) acc -= W(2, i, k) * W(6, i + 1, k);
            if (i + 2 < r1) acc -= W(3, i, k) * W(6, i + 2, k);
            W(6, i, k) = acc / W(1, i, k);
          }
          double nr = 0.0;
          for (int i = r0; i < r1; ++i) nr += W(6, i, k) * W(6, i, k);
          double inv = (nr > 0.0 && nr < 1e300) ? 1.0 / sqrt(nr) : 0.0;
          for (int i = r0; i < r1; ++i) W(5, i, k) = W(6, i, k) * inv;
          // modified Gram-Schmidt against the final vectors near k
          for (int p = na; p < nb && !big; ++p) {
            if (!final_ref(p)) continue;
            double dot = 0.0;
            for (int i = r0; i < r1; ++i) dot += Z(i, p) * W(5, i, k);
            for (int i = r0; i < r1; ++i) W(5, i, k) -= dot * Z(i, p);
          }
          nr = 0.0;
          for (int i = r0; i < r1; ++i) nr += W(5, i, k) * W(5, i, k);
          inv = (nr > 0.0 && nr < 1e300) ? 1.0 / sqrt(nr) : 0.0;
          for (int i = r0; i < r1; ++i) W(5, i, k) *= inv;
        }
        for (int i = 0; i < n; ++i) Z(i, k) = (i >= r0 && i < r1) ? W(5, i, k) : 0.0;
      }
      __syncthreads();
    }
    double* dots = buf + 6144;  // <= 1024 coefficients
    double* gsp = buf + 7168;   // NT partial sums
    int* refs = reinterpret_cast<int*>(buf + 5120);  // <= 1024 reference indices
    // z_j -= sum_t (z_p(t) . z_j) z_p(t), then z_j / |z_j|; passes of
    // classical Gram-Schmidt against nref references: p(t) = ref_base + t,
    // or refs[t] if ref_base < 0.  z_j is staged in LDS (the factors of
    // stages 2-4 are no longer needed); the latency of the global loads, not
    // their number, sets the cost of a call, so the rows of each dot product
    // are split over up to 32 thread groups
    double* zj = buf;
    auto gram_schmidt = [&](int j, int nref, int passes, int ref_base) {
      auto refp = [&](int t) { return ref_base >= 0 ? ref_base + t : refs[t]; };
      for (int pass = 0; pass < passes; ++pass) {
        for (int i = tid; i < n; i += NT) zj[i] = zld(i, j);
        __syncthreads();
        // dots[t] = z_p(t) . z_j, NT references at a time; partial sums in
        // LDS, added in a fixed order
        for (int c0 = 0; c0 < nref; c0 += NT) {
          const int cn = min(NT, nref - c0);
          const int groups = min(max(1, NT / cn), 32);
          const int rows_per = (n + groups - 1) / groups;
          const int t = tid % cn, g = tid / cn;
          if (g < groups) {
            const int p = refp(c0 + t);
            const int i0 = g * rows_per, i1 = min(n, i0 + rows_per);
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int i = i0;
            for (; i + 3 < i1; i += 4) {
              a0 += zld(i, p) * zj[i];
              a1 += zld(i + 1, p) * zj[i + 1];
              a2 += zld(i + 2, p) * zj[i + 2];
              a3 += zld(i + 3, p) * zj[i + 3];
            }
            for (; i < i1; ++i) a0 += zld(i, p) * zj[i];
            gsp[tid] = (a0 + a1) + (a2 + a3);
          }
          __syncthreads();
          for (int tt = tid; tt < cn; tt += NT) {
            double sum = 0.0;
            for (int gg = 0; gg < groups; ++gg) sum += gsp[gg * cn + tt];
            dots[c0 + tt] = sum;
          }
          __syncthreads();
        }
        // z_j -= sum_t dots[t] z_p(t): four lanes per row, combined by
        // shuffles; the row stays in LDS for the normalisation
        double part = 0.0;
        const int q = tid & 3;
        for (int i = tid >> 2; i < n; i += NT >> 2) {
          double s0 = 0.0, s1 = 0.0;
          int t = q;
          for (; t + 4 < nref; t += 8) {
            s0 += dots[t] * zld(i, refp(t));
            s1 += dots[t + 4] * zld(i, refp(t + 4));
          }
          for (; t < nref; t += 4) s0 += dots[t] * zld(i, refp(t));
          double sum = s0 + s1;
          sum += __shfl_xor(sum, 1, 64);
          sum += __shfl_xor(sum, 2, 64);
          const double zi = zj[i] - sum;
          if (q == 0) {
            zj[i] = zi;
            part += zi * zi;
          }
        }
        const double nr = block_sum_dpp(part, red);
        const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
        for (int i = tid; i < n; i += NT) zst(i, j, zj[i] * inv);
        __syncthreads();
      }
    };
    // two block passes of z_(c_lo+c) -= sum_t z_p(t) (z_p(t) . z_(c_lo+c))
    // for the mc columns from c_lo, against the nref references p(t) = ra + t
    // (t < na), rb + t - na (t >= na); coefficients C[t][c] in work array 7
    auto project = [&](int ra, int na, int rb, int nref, int c_lo, int mc) {
      if (nref <= 0 || mc <= 0) return;
      double* C = J.work + (size_t)7 * nc * nc;
      auto ref = [&](int t) { return t < na ? ra + t : rb + (t - na); };
      // 4 x 4 register blocks: eight loads feed sixteen multiply-adds
      const int tb = (nref + 3) >> 2, cb = (mc + 3) >> 2, ib = (n + 3) >> 2;
      for (int pass = 0; pass < 2; ++pass) {
        for (int q = tid; q < tb * cb; q += NT) {
          const int t0 = (q / cb) * 4, c0 = (q % cb) * 4;
          int pt[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) pt[u] = ref(min(t0 + u, nref - 1));
          double acc[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
          for (int i = 0; i < n; ++i) {
            double zp[4], zm[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) zp[u] = zld(i, pt[u]);
#pragma unroll
            for (int v = 0; v < 4; ++v) zm[v] = zld(i, c_lo + min(c0 + v, mc - 1));
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[u][v] = fma(zp[u], zm[v], acc[u][v]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (t0 + u < nref && c0 + v < mc) gstore(C + (size_t)(t0 + u) * nc + c0 + v, acc[u][v]);
        }
        __syncthreads();
        for (int q = tid; q < ib * cb; q += NT) {
          const int i0 = (q / cb) * 4, c0 = (q % cb) * 4;
          double acc[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
          for (int t = 0; t < nref; ++t) {
            const int p = ref(t);
            double zr[4], cv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) zr[u] = zld(min(i0 + u, n - 1), p);
#pragma unroll
            for (int v = 0; v < 4; ++v) cv[v] = gload(C + (size_t)t * nc + min(c0 + v, mc - 1));
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[u][v] = fma(zr[u], cv[v], acc[u][v]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (i0 + u < n && c0 + v < mc) zst(i0 + u, c_lo + c0 + v, zld(i0 + u, c_lo + c0 + v) - acc[u][v]);
        }
        __syncthreads();
      }
    };
    for (int k = 0; k < nres; ++k) {
      if (is_noise(k)) {
        if (k > 0 && is_noise(k - 1)) continue;  // not the start of the noise cluster
        int e = k + 1;
        while (e < nres && is_noise(e)) ++e;
        // the whole cluster at once against every other vector (two block
        // passes), then Gram-Schmidt inside the cluster only
        const int m = e - k;
        project(0, k, e, k + (nres - e), k, m);
        // the members are random vectors already projected off every other
        // vector and well conditioned among themselves: one pass, the block
        // Gram-Schmidt of stage 6 (or the caller's Cholesky pass) removes
        // the second-order overlaps
        for (int j = k; j < e; ++j) gram_schmidt(j, j - k, 1, k);
        continue;
      }
      if (!is_member(k)) continue;
      // references: the vectors of k's block within a relative gap of 1e-3
      // that are final by now (earlier indices, and later ones that are
      // not members); vectors of other blocks are orthogonal by support
      if (tid == 0) {
        int na = k, nb = k + 1;
        while (na > 0 && near(na - 1, k)) --na;
        while (nb < nres && near(nb, k)) ++nb;
        const int bk = s_kb[n - 1 - k];
        int c = 0;
        for (int i = na; i < nb && c < 1024; ++i)
          if (i != k && s_kb[n - 1 - i] == bk && !is_noise(i) && (i < k || !is_member(i))) refs[c++] = i;
        s_nref = c;
      }
      __syncthreads();
      gram_schmidt(k, s_nref, 2, -1);
    }
  }
  __syncthreads();
  stamp(6);
}

// --------------------------------------------------------------- stage 5
// V = Q Z for the selected columns; Q = H_0 H_1 ... H_{n-2}, so the
// reflectors are applied in the order H_{n-2}, ..., H_0.  Each workgroup
// keeps a chunk of HEEV_BT_COLS columns in LDS.  The application is a chain
// of n - 1 dependent steps, so nothing the next step needs from global
// memory waits on the chain: every tau sits in LDS from the start, and the
// next reflector's entries (up to HEEV_BT_PF per lane, which covers n <= 257)
// are loaded into registers while the current one is applied.
constexpr int HEEV_BT_COLS = 8;
constexpr int HEEV_BT_PF = 8;

__global__ void __launch_bounds__(HEEV_THREADS) heev_backtransform_kernel(const HeevJob* jobs) {
  const HeevJob& J = jobs[blockIdx.y];
  const int n = *J.n_ptr;
  if (n > J.n_cap) return;
  const int nvec = (n > 0) ? *J.nvec_out : 0;
  const int c0 = blockIdx.x * HEEV_BT_COLS;
  if (c0 >= nvec) return;
  const int ncol = min(HEEV_BT_COLS, nvec - c0);
  extern __shared__ double2 zs[];  // [HEEV_BT_COLS][n]: a column's lanes read consecutive entries
  __shared__ double2 dots[1][HEEV_BT_COLS];
  __shared__ double2 s_tau[1024];
  const int tid = threadIdx.x;
  const int nc = J.n_cap;
  for (int e = tid; e < n * HEEV_BT_COLS; e += HEEV_THREADS) {
    const int i = e / HEEV_BT_COLS, c = e - i * HEEV_BT_COLS;
    zs[c * n + i] = mk<double>(c < ncol ? J.z[(size_t)i * nc + c0 + c] : 0.0, 0.0);
  }
  const double2* taus = reinterpret_cast<const double2*>(J.tri + 2 * J.n_cap);
  for (int i = tid; i + 1 < n; i += HEEV_THREADS) s_tau[i] = gload(taus + i);
  // 32 lanes per column: thread (c, l) owns rows l, l + 32, ... of column c
  // below the reflector's start, so a column's dot product is one DPP sum
  // over half a wave with no cross-wave sum
  constexpr int LPC = HEEV_THREADS / HEEV_BT_COLS;  // 32
  const int cc = tid / LPC, ll = tid % LPC;
  double2* zc = zs + cc * n;  // this thread's column
  // entries i = ll + LPC t (t < HEEV_BT_PF) of reflector j, zero past its end
  auto fetch = [&](int j, double2* dst) {
    const int m = n - j - 1;
    const double2* v = J.refl + (size_t)max(j, 0) * nc;
#pragma unroll
    for (int t = 0; t < HEEV_BT_PF; ++t) {
      const int i = ll + LPC * t;
      dst[t] = (j >= 0 && i < m) ? gload(v + i) : mk<double>(0.0, 0.0);
    }
  };
  auto apply = [&](int j, const double2* vr) {
    const double2 tau = s_tau[j];
    if (tau.x == 0.0 && tau.y == 0.0) return;
    const int m = n - j - 1;
    const double2* v = J.refl + (size_t)j * nc;
    // s_c = tau * sum_i conj(v_i) z[j+1+i][c]
    double2 part = mk<double>(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < HEEV_BT_PF; ++t) {
      const int i = ll + LPC * t;
      if (i < m) cfmaconj<double>(part, vr[t], zc[j + 1 + i]);
    }
    for (int i = ll + LPC * HEEV_BT_PF; i < m; i += LPC) cfmaconj<double>(part, gload(v + i), zc[j + 1 + i]);
    part.x = half_wave_sum_dpp(part.x);
    part.y = half_wave_sum_dpp(part.y);
    if (ll == LPC - 1) dots[0][cc] = cmul<double>(tau, part);
    __syncthreads();
    const double2 sc = dots[0][cc];
#pragma unroll
    for (int t = 0; t < HEEV_BT_PF; ++t) {
      const int i = ll + LPC * t;
      if (i < m) {
        double2& zz = zc[j + 1 + i];
        zz = csub<double>(zz, cmul<double>(sc, vr[t]));
      }
    }
    for (int i = ll + LPC * HEEV_BT_PF; i < m; i += LPC) {
      double2& zz = zc[j + 1 + i];
      zz = csub<double>(zz, cmul<double>(sc, gload(v + i)));
    }
    __syncthreads();
  };
  double2 va[HEEV_BT_PF], vb[HEEV_BT_PF];
  fetch(n - 2, va);
  __syncthreads();
  for (int j = n - 2; j >= 0; j -= 2) {
    fetch(j - 1, vb);
    apply(j, va);
    if (j - 1 < 0) break;
    fetch(j - 2, va);
    apply(j - 1, vb);
  }
  for (int e = tid; e < n * ncol; e += HEEV_THREADS) {
    const int i = e / ncol, c = e - i * ncol;
    J.v[(size_t)i * J.ldv + c0 + c] = zs[c * n + i];
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
  if (n <= 0 || n > J.n_cap) return;
  const int nvec = *J.nvec_out;
  if (nvec < 2) return;
  // only the strictly upper part of V^H V is used: tiles below the
  // diagonal are skipped
  if (kind == 0 && blockIdx.x > blockIdx.y) return;
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
  if (n <= 0 || n > J.n_cap) return;
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
// last call also applies the column scaling.  64 columns per block (one per
// lane), rows split over the four waves; the partial norms are added in a
// fixed order.  grid (ceil(n_cap / 64), jobs)
__global__ void heev_orth_norm(const HeevJob* jobs, int from_t, int final_pass) {
  const HeevJob& J = jobs[blockIdx.y];
  const int n = *J.n_ptr;
  if (n <= 0 || n > J.n_cap) return;
  const int nvec = *J.nvec_out;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6, ng = blockDim.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  __shared__ double part[4][64];
  const bool use_t = from_t && nvec >= 2;
  const double2* src = use_t ? orth_t(J) : J.v;
  const int lds = use_t ? J.n_cap : J.ldv;
  double acc = 0.0;
  if (k < nvec)
    for (int r = g; r < n; r += ng) acc += cabs2<double>(src[(size_t)r * lds + k]);
  part[g][lane] = acc;
  __syncthreads();
  if (k >= nvec) return;
  double tot = 0.0;
  for (int q = 0; q < ng; ++q) tot += part[q][lane];
  double f = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
  if (final_pass && J.scale != SCALE_NONE) {
    const double lam = fmax(J.w[k], 1e-300);
    f *= (J.scale == SCALE_INV_SQRT) ? 1.0 / sqrt(lam) : sqrt(lam);
  }
  for (int r = g; r < n; r += ng) J.v[(size_t)r * J.ldv + k] = cscale<double>(src[(size_t)r * lds + k], f);
}

}  // namespace ptt
