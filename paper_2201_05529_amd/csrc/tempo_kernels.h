// PT-MPO construction on the GPU: the process-tensor form of the time-
// evolving MPO method (Appendix B.1: window of Delta K_max memory steps,
// relative singular-value threshold eps_TEMPO) for many baths at once.
//
// Influence functional of a Gaussian bath coupled through an operator with
// eigenvalues sigma (Liouville index x = (i, j) -> s+ = sigma_i,
// s- = sigma_j), discretised for piecewise-constant paths:
//   b_Delta(x_k, x_{k-Delta}) = exp(-(s+_k - s-_k)(eta_Delta s+_{k-Delta}
//                                      - conj(eta_Delta) s-_{k-Delta})),
// I = prod_k prod_{Delta=0..min(K, k-1)} b_Delta.
// Step k appends a site carrying b_0, sends x_k leftwards through the last
// K sites while multiplying b_Delta into site k - Delta, and recompresses
// that window: a right-to-left sweep of LQ factorisations (rows made
// orthonormal, no truncation beyond the numerical rank) and a left-to-right
// sweep of truncated SVDs (eps_TEMPO, then the xi cap).  A site that leaves
// the window is final: it is tensor P_j[e][e'][x] of the PT-MPO.
//
// GPU layout: every build is one work item and all builds advance in
// lockstep, step k and window stage i at a time.  Each stage is a short
// sequence of batched launches (Gram matrix, eigensolver, projection,
// rule, push into the neighbouring site), the same pattern as the bond
// update.  The window is a ring of K + 1 site buffers per build.
#pragma once

#include "device_common.h"
#include "gemm_mfma.h"
#include "heev.h"

namespace ptt {

constexpr int TEMPO_D2 = 4;  // Liouville dimension of a spin-1/2 site

enum TempoStage : int { TS_J = 0, TS_ROWS, TS_COLS, TS_N, TS_KEEP, TS_OTHER, TS_ACTIVE, TS_M, TS_COUNT };

struct TempoJob {
  int K, M, xi_cap, acap;      // memory steps, PT-MPO length, bond cap, 4 xi_cap
  double eps;
  const double2* bfac;         // [(K + 1)][16]: b_Delta[x_k][x]
  double2* slots;              // ring [(K + 1)][acap * 4 * acap], site tensor [a][x][c]
  int* sa;                     // [K + 1] left dims of the ring slots
  int* sc;                     // [K + 1] right dims
  double2* tmp;                // [acap * 4 * acap]
  double2* g;                  // [acap * acap] Gram matrix, then L or S V^H
  double2* w;                  // [acap * acap] eigenvectors
  double2* p;                  // [4 acap * acap] projection
  double* lam;                 // [acap] eigenvalues
  double* s;                   // [acap] norms
  int* perm;                   // [acap] order of the norms
  int* sd;                     // [TS_COUNT] stage dims
  double2* out;                // [M][xi_cap * xi_cap * 4] P_k[e][e'][x]
  int* out_dims;               // [M + 1]
  int* status;                 // heev status word
};

__device__ inline double2* tempo_slot(const TempoJob& J, int site) {
  return J.slots + (long long)(site % (J.K + 1)) * J.acap * TEMPO_D2 * J.acap;
}

// The site of step f leaves the window: P_f[e][e'][x] = t[e][x][e'].
__device__ inline void tempo_freeze(const TempoJob& J, int f) {
  const int pos = f % (J.K + 1);
  const int a = J.sa[pos], c = J.sc[pos];
  const double2* t = tempo_slot(J, f);
  double2* o = J.out + (long long)(f - 1) * J.xi_cap * J.xi_cap * TEMPO_D2;
  for (int idx = threadIdx.x; idx < a * TEMPO_D2 * c; idx += blockDim.x) {
    const int cc = idx % c, rest = idx / c;
    const int x = rest % TEMPO_D2, aa = rest / TEMPO_D2;
    o[((long long)aa * c + cc) * TEMPO_D2 + x] = t[idx];
  }
  if (threadIdx.x == 0) {
    J.out_dims[f - 1] = a;
    J.out_dims[f] = c;
  }
}

// Step k, before the recompression: freeze the site leaving the window,
// append site k, emit x_k on a new left bond of site k and multiply b_Delta
// into the window sites (the bonds they carry x_k through grow by d^2).
// One block per build.
__global__ void k_tempo_begin(const TempoJob* jobs, int k) {
  const TempoJob& J = jobs[blockIdx.x];
  const int K = J.K;
  if (k > J.M) {
    if (threadIdx.x == 0) J.sd[TS_ACTIVE] = 0;
    return;
  }
  if (k - K - 1 >= 1) tempo_freeze(J, k - K - 1);
  __syncthreads();
  const int m = min(K, k - 1);
  const int pos = k % (K + 1);
  double2* t = tempo_slot(J, k);
  // site k: b_0 on the diagonal; with m >= 1 its index goes out on the left
  if (m == 0) {
    if (threadIdx.x < TEMPO_D2) t[threadIdx.x] = J.bfac[threadIdx.x * TEMPO_D2 + threadIdx.x];
    if (threadIdx.x == 0) { J.sa[pos] = 1; J.sc[pos] = 1; }
  } else {
    // [a = x_e][x][c = 1]: delta(x_e, x) b_0[x][x]
    if (threadIdx.x < TEMPO_D2 * TEMPO_D2) {
      const int xe = threadIdx.x / TEMPO_D2, x = threadIdx.x % TEMPO_D2;
      t[threadIdx.x] = xe == x ? J.bfac[x * TEMPO_D2 + x] : mk<double>(0.0, 0.0);
    }
    if (threadIdx.x == 0) { J.sa[pos] = TEMPO_D2; J.sc[pos] = 1; }
  }
  __syncthreads();
  for (int dl = 1; dl <= m; ++dl) {
    const int site = k - dl, sp = site % (K + 1);
    const bool through = dl < m;
    const int a = J.sa[sp], c = J.sc[sp];
    const int na = through ? a * TEMPO_D2 : a, nc = c * TEMPO_D2;
    const double2* src = tempo_slot(J, site);
    const double2* bf = J.bfac + dl * 16;
    for (int idx = threadIdx.x; idx < na * TEMPO_D2 * nc; idx += blockDim.x) J.tmp[idx] = mk<double>(0.0, 0.0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < a * TEMPO_D2 * c * TEMPO_D2; idx += blockDim.x) {
      const int xk = idx % TEMPO_D2, r1 = idx / TEMPO_D2;
      const int cc = r1 % c, r2 = r1 / c;
      const int x = r2 % TEMPO_D2, aa = r2 / TEMPO_D2;
      const int oa = through ? aa * TEMPO_D2 + xk : aa;
      J.tmp[((long long)oa * TEMPO_D2 + x) * nc + cc * TEMPO_D2 + xk] =
          cmul<double>(src[((long long)aa * TEMPO_D2 + x) * c + cc], bf[xk * TEMPO_D2 + x]);
    }
    __syncthreads();
    double2* dst = tempo_slot(J, site);
    for (int idx = threadIdx.x; idx < na * TEMPO_D2 * nc; idx += blockDim.x) dst[idx] = J.tmp[idx];
    __syncthreads();
    if (threadIdx.x == 0) { J.sa[sp] = na; J.sc[sp] = nc; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    J.sd[TS_ACTIVE] = 1;
    J.sd[TS_M] = m;
  }
}

// Stage set-up, one thread per build.  rl = 1: site j = k - i, matrix
// a x (d^2 c), Gram over rows; rl = 0: site j = k - m + i, matrix
// (a d^2) x c, Gram over columns.  N = 0 switches the stage off.
__global__ void k_tempo_stage(const TempoJob* jobs, int n_jobs, int k, int i, int rl) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_jobs) return;
  const TempoJob& J = jobs[b];
  int* sd = J.sd;
  const int m = sd[TS_M];
  if (!sd[TS_ACTIVE] || i >= m) {  // every count the stage's kernels read becomes zero
    sd[TS_N] = 0;
    sd[TS_ROWS] = 0;
    sd[TS_COLS] = 0;
    sd[TS_KEEP] = 0;
    return;
  }
  const int j = rl ? k - i : k - m + i;
  const int pos = j % (J.K + 1);
  sd[TS_J] = j;
  if (rl) {
    sd[TS_ROWS] = J.sa[pos];
    sd[TS_COLS] = TEMPO_D2 * J.sc[pos];
    sd[TS_N] = sd[TS_ROWS];
  } else {
    sd[TS_ROWS] = TEMPO_D2 * J.sa[pos];
    sd[TS_COLS] = J.sc[pos];
    sd[TS_N] = sd[TS_COLS];
  }
}

enum TempoGemm : int { TG_RL_GRAM = 0, TG_RL_PROJ, TG_RL_PUSH, TG_LR_GRAM, TG_LR_PROJ, TG_LR_PUSH };

__device__ inline bool tempo_gemm_args(const TempoJob& J, int kind, GemmArgs& g) {
  const int* sd = J.sd;
  if (sd[TS_N] == 0) return false;
  const int j = sd[TS_J], rows = sd[TS_ROWS], cols = sd[TS_COLS], keep = sd[TS_KEEP];
  const int acap = J.acap;
  g.alpha = 1.0;
  g.acc = false;
  auto set = [&](const double2* A, int lda, bool ca, const double2* B, int ldb, bool cb, double2* C, int ldc,
                 int m, int n, int kk) {
    g.A = A; g.lda = lda; g.ca = ca; g.B = B; g.ldb = ldb; g.cb = cb; g.C = C; g.ldc = ldc;
    g.m = m; g.n = n; g.k = kk;
  };
  const double2* M = tempo_slot(J, j);
  switch (kind) {
    case TG_RL_GRAM:  // g = M M^H
      set(M, cols, false, M, cols, true, J.g, acap, rows, rows, cols);
      return true;
    case TG_RL_PROJ:  // p = W^H M (keep x cols)
      set(J.w, acap, true, M, cols, false, J.p, cols, keep, cols, rows);
      return true;
    case TG_RL_PUSH: {  // tmp = site_{j-1} (d^2 a' x rows) L (rows x keep)
      const int pp = (j - 1) % (J.K + 1);
      const double2* S = tempo_slot(J, j - 1);
      set(S, rows, false, J.g, acap, false, J.tmp, keep, TEMPO_D2 * J.sa[pp], keep, rows);
      return true;
    }
    case TG_LR_GRAM:  // g = M^H M
      set(M, cols, true, M, cols, false, J.g, acap, cols, cols, rows);
      return true;
    case TG_LR_PROJ:  // p = M W (rows x cols)
      set(M, cols, false, J.w, acap, false, J.p, cols, rows, cols, cols);
      return true;
    case TG_LR_PUSH: {  // tmp = (S V^H) (keep x cols) site_{j+1} (cols x d^2 c')
      const int pn = (j + 1) % (J.K + 1);
      const int w2 = TEMPO_D2 * J.sc[pn];
      set(J.g, acap, false, tempo_slot(J, j + 1), w2, false, J.tmp, w2, keep, w2, cols);
      return true;
    }
  }
  return false;
}

// grid (tiles_m, tiles_n, builds)
__global__ void __launch_bounds__(GEMM_THREADS) k_tempo_gemm(const TempoJob* jobs, int kind) {
  __shared__ MfmaSmem<double> sm;
  GemmArgs g;
  if (!tempo_gemm_args(jobs[blockIdx.z], kind, g)) return;
  if (g.m <= 0 || g.n <= 0) return;
  gemm_tile_mfma<double>(g.A, g.lda, g.ca, g.B, g.ldb, g.cb, g.C, g.ldc, g.m, g.n, g.k,
                         mk<double>(g.alpha, 0.0), g.acc, blockIdx.x, blockIdx.y, sm);
}

// R -> L: the rows of p = W^H M (W unitary, so M = W p) with norms s,
// ordered by norm, become the new site j (orthonormal rows); rows whose norm
// is below 1e-14 of the largest are the numerical null space of M and are
// dropped.  L = W diag(s) (rows x keep) goes to g for the push.  One block
// per build.
constexpr double TEMPO_RANK_TOL = 1e-14;

__global__ void k_tempo_rl_finish(const TempoJob* jobs) {
  const TempoJob& J = jobs[blockIdx.x];
  int* sd = J.sd;
  if (sd[TS_N] == 0) return;
  const int j = sd[TS_J], rows = sd[TS_ROWS], cols = sd[TS_COLS], n = sd[TS_KEEP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r = wv; r < n; r += nw) {
    double acc = 0.0;
    for (int c = lane; c < cols; c += 64) acc += cabs2<double>(J.p[(long long)r * cols + c]);
    acc = warp_sum(acc);
    if (lane == 0) J.s[r] = sqrt(acc);
  }
  __syncthreads();
  // descending order (equal norms by index): perm[rank] = row
  __shared__ double s_max;
  __shared__ int s_keep;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const double v = J.s[r];
    int rank = 0;
    for (int q = 0; q < n; ++q) {
      const double u = J.s[q];
      rank += (u > v) || (u == v && q < r);
    }
    J.perm[rank] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_max = n > 0 ? J.s[J.perm[0]] : 0.0;
    int keep = 0;
    while (keep < n && J.s[J.perm[keep]] > TEMPO_RANK_TOL * s_max) ++keep;
    s_keep = max(keep, 1);
  }
  __syncthreads();
  const int keep = s_keep;
  double2* M = tempo_slot(J, j);
  for (int idx = threadIdx.x; idx < keep * cols; idx += blockDim.x) {
    const int r = idx / cols, c = idx - r * cols;
    const int src = J.perm[r];
    const double sr = J.s[src];
    M[idx] = sr > 0.0 ? cscale<double>(J.p[(long long)src * cols + c], 1.0 / sr) : mk<double>(0.0, 0.0);
  }
  for (int idx = threadIdx.x; idx < rows * keep; idx += blockDim.x) {
    const int r = idx / keep, c = idx % keep;
    const int src = J.perm[c];
    J.g[(long long)r * J.acap + c] = cscale<double>(J.w[(long long)r * J.acap + src], J.s[src]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    J.sa[j % (J.K + 1)] = keep;
    sd[TS_KEEP] = keep;
  }
}

// L -> R: singular values are the norms of the columns of p = M W, sorted;
// the smallest rank whose discarded tail has 2-norm below eps times the
// largest (zeros never kept, rank >= 1), then the xi cap.  U = p S^-1 becomes
// site j (right dim keep); S V^H (keep x cols) goes to g for the push.
// One block per build.
__global__ void k_tempo_lr_rule(const TempoJob* jobs) {
  const TempoJob& J = jobs[blockIdx.x];
  int* sd = J.sd;
  if (sd[TS_N] == 0) return;
  const int j = sd[TS_J], rows = sd[TS_ROWS], cols = sd[TS_COLS];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wv; c < cols; c += nw) {
    double acc = 0.0;
    for (int r = lane; r < rows; r += 64) acc += cabs2<double>(J.p[(long long)r * cols + c]);
    acc = warp_sum(acc);
    if (lane == 0) J.s[c] = sqrt(acc);
  }
  __syncthreads();
  __shared__ int s_keep;
  if (threadIdx.x == 0) {
    for (int c = 0; c < cols; ++c) J.perm[c] = c;
    for (int a = 1; a < cols; ++a) {  // insertion sort, descending norms (stable)
      const int v = J.perm[a];
      int b = a - 1;
      while (b >= 0 && J.s[J.perm[b]] < J.s[v]) {
        J.perm[b + 1] = J.perm[b];
        --b;
      }
      J.perm[b + 1] = v;
    }
    int npos = 0;
    while (npos < cols && J.s[J.perm[npos]] > 0.0) ++npos;
    int keep = max(npos, 1);
    if (npos > 0) {
      const double thr = J.eps * J.s[J.perm[0]];
      double tail = 0.0;
      for (int c = npos - 1; c >= 1; --c) {
        tail += J.s[J.perm[c]] * J.s[J.perm[c]];
        if (sqrt(tail) < thr) keep = c;
        else break;
      }
    }
    keep = min(keep, J.xi_cap);
    s_keep = keep;
    sd[TS_KEEP] = keep;
  }
  __syncthreads();
  const int keep = s_keep;
  // U into the site buffer through tmp (p and the site are distinct buffers)
  double2* M = tempo_slot(J, j);
  for (int idx = threadIdx.x; idx < rows * keep; idx += blockDim.x) {
    const int r = idx / keep, c = idx % keep;
    const int src = J.perm[c];
    const double sv = J.s[src];
    M[idx] = sv > 0.0 ? cscale<double>(J.p[(long long)r * cols + src], 1.0 / sv) : mk<double>(0.0, 0.0);
  }
  for (int idx = threadIdx.x; idx < keep * cols; idx += blockDim.x) {
    const int r = idx / cols, c = idx % cols;
    const int src = J.perm[r];
    J.g[(long long)r * J.acap + c] = cscale<double>(cconj<double>(J.w[(long long)c * J.acap + src]), J.s[src]);
  }
  __syncthreads();
  if (threadIdx.x == 0) J.sc[j % (J.K + 1)] = keep;
}

// the pushed product back into the neighbouring site.  rl = 1: site j - 1
// gets right dim keep; rl = 0: site j + 1 gets left dim keep.  One block per
// build.
__global__ void k_tempo_push_copy(const TempoJob* jobs, int rl) {
  const TempoJob& J = jobs[blockIdx.x];
  const int* sd = J.sd;
  if (sd[TS_N] == 0) return;
  const int j = sd[TS_J], keep = sd[TS_KEEP];
  const int nb = rl ? j - 1 : j + 1;
  const int pos = nb % (J.K + 1);
  const long long tot = rl ? (long long)TEMPO_D2 * J.sa[pos] * keep : (long long)keep * TEMPO_D2 * J.sc[pos];
  double2* dst = tempo_slot(J, nb);
  for (long long idx = threadIdx.x; idx < tot; idx += blockDim.x) dst[idx] = J.tmp[idx];
  __syncthreads();
  if (threadIdx.x == 0) {
    if (rl) J.sc[pos] = keep;
    else J.sa[pos] = keep;
  }
}

// after the last step: the sites still in the window are final.  One block
// per build.
__global__ void k_tempo_end(const TempoJob* jobs) {
  const TempoJob& J = jobs[blockIdx.x];
  for (int f = max(1, J.M - J.K); f <= J.M; ++f) {
    tempo_freeze(J, f);
    __syncthreads();
  }
}

}  // namespace ptt
