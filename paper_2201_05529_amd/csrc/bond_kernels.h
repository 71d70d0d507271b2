// Kernels of one Trotter sublayer of PT-TEBD: every bond update of the
// sublayer (and, for batched runs, of every chain) is one work item; each
// phase below is one launch over all items.  All dimensions live in device
// memory, so the launch sequence is fixed and is enqueued without host
// synchronisation.
//
// Two-site update, Appendix A.2 (c)-(h), with the truncated SVDs computed
// through Gram matrices and a double-precision Hermitian eigensolver:
//   pack      B_L = lam_{n-1} Gamma_n as (a,e) x (s,b);  B_R = Gamma_{n+1} lam_{n+1}
//             as (b,t) x (f,c)                                          (c)-(d)
//   gram      G_L, G_R on the smaller side of each matrix
//   heev      eigenpairs; the eps rule gives the ranks l, r             (d)-(e)
//   xy        X = S_L V_L^H (l x (s,b)) times lam_n on b;  Y = U_R S_R
//   p, gate   P[(l,s),(t,r)] = sum_b X Y;  D = G applied on (s,t)       (e)-(f)
//   rf        randomised range finder for the leading singular subspace of D
//             (Gaussian sketch, power iteration, orthonormalisation by the
//             eigendecomposition of the basis Gram matrix), Rayleigh-Ritz on
//             Q^H D with the eps rule, the chi_max cap and the tie rule  (f)-(g)
//   rebuild   Gamma_n' = lam_{n-1}^-1 U_L U^D,  Gamma_{n+1}' = V^D^H V_R^H
//             lam_{n+1}^-1; where the eigenvectors sit on the far side of B
//             the same products are evaluated as B V S^-1 U^D (resp.
//             V^D^H S^-1 U^H B), which is the identical algebra  (g)-(h)
//   finalize  new bond vector S^D / ||S^D||_2, log-scale += log ||S^D||_2
#pragma once

#include "device_common.h"
#include "gemm.h"
#include "heev.h"

namespace ptt {

// -------------------------------------------------------------- state
struct ChainDev {
  int n_sites, chi_cap, xi_cap, pad;
  long long gam_cap;     // complex elements per Gamma buffer
  double2* gam;          // [n_sites][2][gam_cap], Gamma[a][s][e][b] compact
  int* parity;           // [n_sites] which of the two buffers is current
  int* chi;              // [n_sites + 1] bond dims, chi[0] = chi[N] = 1
  int* xi;               // [n_sites] augmented-leg dims
  double* lam;           // [(n_sites + 1) * chi_cap]
  double* log_scale;     // [1]
  int* status;           // [1] sticky error bits
};

__device__ inline double2* gamma_cur(const ChainDev& c, int site) {
  return c.gam + ((long long)site * 2 + c.parity[site]) * c.gam_cap;
}
__device__ inline double2* gamma_next(const ChainDev& c, int site) {
  return c.gam + ((long long)site * 2 + (1 - c.parity[site])) * c.gam_cap;
}

enum Dim : int {
  D_A = 0, D_E, D_B, D_F, D_C,
  D_RL, D_CL, D_NL, D_SL,      // B_L rows, cols, Gram size, side (0: B^H B, 1: B B^H)
  D_RR, D_CR, D_NR, D_SR,      // B_R rows, cols, Gram size, side (0: B B^H, 1: B^H B)
  D_L, D_R, D_M, D_N,          // ranks l, r; D is M x N = 4l x 4r
  D_K, D_KQ, D_KZ, D_GS,       // sketch width, basis widths, current Gram size
  D_CHI,                       // new bond dimension
  D_COUNT
};

enum StatusBits : int { ST_NONFINITE = 1, ST_ZERO = 2, ST_EIG = 4, ST_RANGE = 8 };

struct BondJob {
  int chain;               // index into the chain array passed to the kernels
  int bond;                // sites bond, bond+1
  const double2* gate;     // [16][16] site-major
  int chi_max;
  int k_cap;               // sketch width cap
  double eps;
  unsigned long long seed;
  int nb_cap;              // capacity of B Gram sizes (4 chi_cap); ld of gl/gr/vl/vr
  int dn_cap;              // capacity of M, N (4 nb_cap)
  int* dims;               // [D_COUNT]
  double* norms;           // [4]: ||D||_F^2, ||Q^H D||_F^2, extra tail, spare
  double2 *bl, *br, *gl, *gr, *vl, *vr, *x, *y, *p, *d;
  double *wl, *wr, *wk;
  double2 *omega, *ya, *yb, *za, *zb, *gk, *vk, *bm, *ud, *vdh, *t1, *tg;
};

// ------------------------------------------------------------------ pack
// grid (blocks, items)
__global__ void k_pack(const ChainDev* chains, const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  const ChainDev& C = chains[J.chain];
  const int a = C.chi[J.bond], e = C.xi[J.bond], b = C.chi[J.bond + 1];
  const int f = C.xi[J.bond + 1], c = C.chi[J.bond + 2];
  const int rl = a * e, cl = 4 * b, rr = 4 * b, cr = f * c;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int* D = J.dims;
    D[D_A] = a; D[D_E] = e; D[D_B] = b; D[D_F] = f; D[D_C] = c;
    D[D_RL] = rl; D[D_CL] = cl; D[D_SL] = (cl <= rl) ? 0 : 1; D[D_NL] = min(rl, cl);
    D[D_RR] = rr; D[D_CR] = cr; D[D_SR] = (rr <= cr) ? 0 : 1; D[D_NR] = min(rr, cr);
    for (int i = 0; i < 4; ++i) J.norms[i] = 0.0;
  }
  const double2* gl = gamma_cur(C, J.bond);
  const double2* gr = gamma_cur(C, J.bond + 1);
  const double* lam_l = C.lam + (long long)J.bond * C.chi_cap;
  const double* lam_r = C.lam + (long long)(J.bond + 2) * C.chi_cap;
  const long long nl = (long long)rl * cl, nr = (long long)rr * cr;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nl + nr;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < nl) {
      const int row = (int)(idx / cl), col = (int)(idx - (long long)row * cl);
      const int ai = row / e, ei = row - ai * e;
      const int s = col / b, bi = col - s * b;
      const double2 g = gl[((long long)(ai * 4 + s) * e + ei) * b + bi];
      J.bl[idx] = cscale<double>(g, lam_l[ai]);
    } else {
      const long long j = idx - nl;
      J.br[j] = cscale<double>(gr[j], lam_r[(int)(j % c)]);
    }
  }
}

// ------------------------------------------------------- batched products
enum GemmKind : int {
  GK_GRAM_B = 0,   // sub 0: G_L, sub 1: G_R
  GK_XY,           // sub 0: X = U_L^H B_L (rows side), sub 1: Y = B_R V_R (cols side)
  GK_P,            // P = X' Y'
  GK_SKETCH,       // ya = D omega                     (M x K)
  GK_GRAM_YA,      // gk = ya^H ya                     (GS x GS)
  GK_APPLY_YA,     // yb = ya vk                       (M x KQ)
  GK_GRAM_YB,      // gk = yb^H yb
  GK_APPLY_YB,     // ya = yb vk                       (M x KQ)
  GK_DH_Q,         // za = D^H ya                      (N x KQ)
  GK_GRAM_ZA,      // gk = za^H za
  GK_APPLY_ZA,     // zb = za vk                       (N x KZ)
  GK_GRAM_ZB,      // gk = zb^H zb
  GK_APPLY_ZB,     // za = zb vk                       (N x KZ)
  GK_D_Z,          // ya = D za                        (M x KZ)
  GK_QH_D,         // bm = ya^H D                      (KQ x N)
  GK_GRAM_BM,      // gk = bm bm^H                     (KQ x KQ)
  GK_UD,           // ud = ya vk                       (M x CHI)
  GK_VDH,          // vdh = vk^H bm                    (CHI x N)
  GK_T1,           // side-0 left: t1 = V_L (S^-1 U^D')
  GK_NEWL,         // tg = B_L t1 (side 0) or U_L U^D' (side 1)
  GK_T2,           // side-0 right: t1 = (V^D' S^-1) U_R^H
  GK_NEWR,         // tg = t1 B_R (side 0) or V^D' V_R^H (side 1)
};

struct GemmArgs {
  const double2* A; int lda; bool ca;
  const double2* B; int ldb; bool cb;
  double2* C; int ldc;
  int m, n, k;
};

__device__ inline bool gemm_args(const BondJob& J, int kind, int sub, GemmArgs& g) {
  const int* D = J.dims;
  const int kc = J.k_cap, nb = J.nb_cap;
  switch (kind) {
    case GK_GRAM_B:
      if (sub == 0) {
        const int rl = D[D_RL], cl = D[D_CL];
        if (D[D_SL] == 0) g = {J.bl, cl, true, J.bl, cl, false, J.gl, nb, cl, cl, rl};
        else g = {J.bl, cl, false, J.bl, cl, true, J.gl, nb, rl, rl, cl};
      } else {
        const int rr = D[D_RR], cr = D[D_CR];
        if (D[D_SR] == 0) g = {J.br, cr, false, J.br, cr, true, J.gr, nb, rr, rr, cr};
        else g = {J.br, cr, true, J.br, cr, false, J.gr, nb, cr, cr, rr};
      }
      return true;
    case GK_XY:
      if (sub == 0) {
        if (D[D_SL] != 1) return false;
        g = {J.vl, nb, true, J.bl, D[D_CL], false, J.x, D[D_CL], D[D_L], D[D_CL], D[D_RL]};
      } else {
        if (D[D_SR] != 1) return false;
        g = {J.br, D[D_CR], false, J.vr, nb, false, J.y, D[D_R], D[D_RR], D[D_R], D[D_CR]};
      }
      return true;
    case GK_P:
      g = {J.x, D[D_B], false, J.y, 4 * D[D_R], false, J.p, 4 * D[D_R], 4 * D[D_L], 4 * D[D_R], D[D_B]};
      return true;
    case GK_SKETCH:
      g = {J.d, D[D_N], false, J.omega, kc, false, J.ya, kc, D[D_M], D[D_K], D[D_N]};
      return true;
    case GK_GRAM_YA:
      g = {J.ya, kc, true, J.ya, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_M]};
      return true;
    case GK_APPLY_YA:
      g = {J.ya, kc, false, J.vk, kc, false, J.yb, kc, D[D_M], D[D_KQ], D[D_GS]};
      return true;
    case GK_GRAM_YB:
      g = {J.yb, kc, true, J.yb, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_M]};
      return true;
    case GK_APPLY_YB:
      g = {J.yb, kc, false, J.vk, kc, false, J.ya, kc, D[D_M], D[D_KQ], D[D_GS]};
      return true;
    case GK_DH_Q:
      g = {J.d, D[D_N], true, J.ya, kc, false, J.za, kc, D[D_N], D[D_KQ], D[D_M]};
      return true;
    case GK_GRAM_ZA:
      g = {J.za, kc, true, J.za, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_N]};
      return true;
    case GK_APPLY_ZA:
      g = {J.za, kc, false, J.vk, kc, false, J.zb, kc, D[D_N], D[D_KZ], D[D_GS]};
      return true;
    case GK_GRAM_ZB:
      g = {J.zb, kc, true, J.zb, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_N]};
      return true;
    case GK_APPLY_ZB:
      g = {J.zb, kc, false, J.vk, kc, false, J.za, kc, D[D_N], D[D_KZ], D[D_GS]};
      return true;
    case GK_D_Z:
      g = {J.d, D[D_N], false, J.za, kc, false, J.ya, kc, D[D_M], D[D_KZ], D[D_N]};
      return true;
    case GK_QH_D:
      g = {J.ya, kc, true, J.d, D[D_N], false, J.bm, D[D_N], D[D_KQ], D[D_N], D[D_M]};
      return true;
    case GK_GRAM_BM:
      g = {J.bm, D[D_N], false, J.bm, D[D_N], true, J.gk, kc, D[D_KQ], D[D_KQ], D[D_N]};
      return true;
    case GK_UD:
      g = {J.ya, kc, false, J.vk, kc, false, J.ud, D[D_CHI], D[D_M], D[D_CHI], D[D_KQ]};
      return true;
    case GK_VDH:
      g = {J.vk, kc, true, J.bm, D[D_N], false, J.vdh, D[D_N], D[D_CHI], D[D_N], D[D_KQ]};
      return true;
    case GK_T1:  // side 0: t1 (cl x 4chi) = V_L (cl x l) ud' (l x 4chi)
      if (D[D_SL] != 0) return false;
      g = {J.vl, nb, false, J.ud, 4 * D[D_CHI], false, J.t1, 4 * D[D_CHI], D[D_CL], 4 * D[D_CHI], D[D_L]};
      return true;
    case GK_NEWL:
      if (D[D_SL] == 0)  // tg (rl x 4chi) = B_L (rl x cl) t1
        g = {J.bl, D[D_CL], false, J.t1, 4 * D[D_CHI], false, J.tg, 4 * D[D_CHI], D[D_RL], 4 * D[D_CHI], D[D_CL]};
      else               // tg = U_L (rl x l) ud' (l x 4chi)
        g = {J.vl, nb, false, J.ud, 4 * D[D_CHI], false, J.tg, 4 * D[D_CHI], D[D_RL], 4 * D[D_CHI], D[D_L]};
      return true;
    case GK_T2:  // side 0: t1 (4chi x rr) = vdh' (4chi x r) U_R^H (r x rr)
      if (D[D_SR] != 0) return false;
      g = {J.vdh, D[D_R], false, J.vr, nb, true, J.t1, D[D_RR], 4 * D[D_CHI], D[D_RR], D[D_R]};
      return true;
    case GK_NEWR:
      if (D[D_SR] == 0)  // tg (4chi x cr) = t1 (4chi x rr) B_R (rr x cr)
        g = {J.t1, D[D_RR], false, J.br, D[D_CR], false, J.tg, D[D_CR], 4 * D[D_CHI], D[D_CR], D[D_RR]};
      else               // tg = vdh' (4chi x r) V_R^H (r x cr)
        g = {J.vdh, D[D_R], false, J.vr, nb, true, J.tg, D[D_CR], 4 * D[D_CHI], D[D_CR], D[D_R]};
      return true;
    default:
      return false;
  }
}

// grid (tiles_m, tiles_n, items * subs)
__global__ void __launch_bounds__(GEMM_THREADS) k_bond_gemm(const BondJob* jobs, int kind, int subs) {
  __shared__ GemmSmem<double> sm;
  const int item = blockIdx.z / subs, sub = blockIdx.z - item * subs;
  GemmArgs g;
  if (!gemm_args(jobs[item], kind, sub, g)) return;
  if (g.m <= 0 || g.n <= 0) return;
  gemm_tile<double>(g.A, g.lda, g.ca, g.B, g.ldb, g.cb, g.C, g.ldc, g.m, g.n, g.k,
                    mk<double>(1.0, 0.0), false, blockIdx.x, blockIdx.y, sm);
}

// ------------------------------------------------------ X, Y (elementwise)
// X (l x cl): side 0 -> S_L V_L^H; side 1 -> GEMM result already in x.  Both
// then scaled by lam_n on the b index.  Y (rr x r): side 0 -> U_R S_R.
// grid (blocks, items)
__global__ void k_form_xy(const ChainDev* chains, const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  const ChainDev& C = chains[J.chain];
  const int* D = J.dims;
  const int l = D[D_L], r = D[D_R], cl = D[D_CL], rr = D[D_RR], b = D[D_B];
  const double* lam_c = C.lam + (long long)(J.bond + 1) * C.chi_cap;
  const int nb = J.nb_cap;
  const long long nx = (long long)l * cl, ny = (long long)rr * r;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nx + ny;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < nx) {
      const int i = (int)(idx / cl), col = (int)(idx - (long long)i * cl);
      const double lb = lam_c[col % b];
      double2 v;
      if (D[D_SL] == 0) {
        const double s = sqrt(fmax(J.wl[i], 0.0));
        v = cscale<double>(cconj<double>(J.vl[(long long)col * nb + i]), s);
      } else {
        v = J.x[idx];
      }
      J.x[idx] = cscale<double>(v, lb);
    } else if (D[D_SR] == 0) {
      const long long j = idx - nx;
      const int row = (int)(j / r), k = (int)(j - (long long)row * r);
      const double s = sqrt(fmax(J.wr[k], 0.0));
      J.y[j] = cscale<double>(J.vr[(long long)row * nb + k], s);
    }
  }
}

// ------------------------------------------------------------ gate on P
// D[(l,s'),(t',r)] = sum_{s,t} G[(s',t'),(s,t)] P[(l,s),(t,r)]; also sets
// M, N and the sketch width, accumulates ||D||_F^2.  grid (blocks, items)
__global__ void k_apply_gate(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  int* D = J.dims;
  const int l = D[D_L], r = D[D_R];
  const int M = 4 * l, N = 4 * r;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D[D_M] = M;
    D[D_N] = N;
    const int k = min(min(M, N), J.k_cap);
    D[D_K] = k;
    D[D_GS] = k;
  }
  __shared__ double2 g[256];
  __shared__ double red[4];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) g[i] = J.gate[i];
  __syncthreads();
  double part = 0.0;
  const long long npairs = (long long)l * r;
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < npairs;
       pr += (long long)gridDim.x * blockDim.x) {
    const int li = (int)(pr / r), ri = (int)(pr - (long long)li * r);
    double2 in[16];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) in[s * 4 + t] = J.p[(long long)(li * 4 + s) * N + t * r + ri];
#pragma unroll
    for (int so = 0; so < 4; ++so)
#pragma unroll
      for (int to = 0; to < 4; ++to) {
        double2 acc = mk<double>(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 16; ++q) cfma<double>(acc, g[(so * 4 + to) * 16 + q], in[q]);
        J.d[(long long)(li * 4 + so) * N + to * r + ri] = acc;
        part += cabs2<double>(acc);
      }
  }
  const double tot = block_sum(part, red);
  if (threadIdx.x == 0 && tot != 0.0) atomicAdd(&J.norms[0], tot);
}

// ------------------------------------------------------ range finder init
// Gaussian sketch omega (N x K), counter-based (SplitMix64 + Box-Muller).
__global__ void k_sketch_init(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  const int N = J.dims[D_N], K = J.dims[D_K];
  const long long tot = (long long)N * K;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int row = (int)(idx / K), col = (int)(idx - (long long)row * K);
    const unsigned long long ctr = J.seed ^ (0x9E3779B97F4A7C15ull * (unsigned long long)(row * 4099 + col + 1));
    const double u1 = u01(splitmix64(ctr)), u2 = u01(splitmix64(ctr ^ 0xD1B54A32D192ED03ull));
    const double rad = sqrt(-2.0 * log(u1));
    J.omega[(long long)row * J.k_cap + col] = mk<double>(rad * cos(6.283185307179586 * u2),
                                                        rad * sin(6.283185307179586 * u2));
  }
}

// small dims bookkeeping kernel: dims[dst] = dims[src] for every item
__global__ void k_copy_dim(const BondJob* jobs, int n_items, int dst, int src) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_items) jobs[i].dims[dst] = jobs[i].dims[src];
}

// ||Q^H D||_F^2 -> norms[1]; extra tail = max(||D||^2 - ||Q^H D||^2, 0) -> norms[2]
__global__ void k_rr_norms(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.x];
  const int kq = J.dims[D_KQ], N = J.dims[D_N];
  __shared__ double red[4];
  double part = 0.0;
  for (long long idx = threadIdx.x; idx < (long long)kq * N; idx += blockDim.x) part += cabs2<double>(J.bm[idx]);
  const double tot = block_sum(part, red);
  if (threadIdx.x == 0) {
    J.norms[1] = tot;
    J.norms[2] = fmax(J.norms[0] - tot, 0.0);
  }
}

// rows of vdh /= sigma_i (V^D^H = S^-1 W^H B); side-0 scalings used by the
// rebuilds: ud rows (l,s') /= sigma_L[l], vdh' columns r /= sigma_R[r].
__global__ void k_scale_factors(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  const int* D = J.dims;
  const int chi = D[D_CHI], N = D[D_N], M = D[D_M], r = D[D_R];
  const long long nv = (long long)chi * N, nu = (long long)M * chi;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nv + nu;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < nv) {
      const int i = (int)(idx / N), col = (int)(idx - (long long)i * N);
      double f = 1.0 / sqrt(fmax(J.wk[i], 1e-300));
      if (D[D_SR] == 0) f /= sqrt(fmax(J.wr[col % r], 1e-300));
      J.vdh[idx] = cscale<double>(J.vdh[idx], f);
    } else if (D[D_SL] == 0) {
      const long long j = idx - nv;
      const int row = (int)(j / chi);
      J.ud[j] = cscale<double>(J.ud[j], 1.0 / sqrt(fmax(J.wl[row / 4], 1e-300)));
    }
  }
}

// ---------------------------------------------------------------- stores
// New Gamma_n[a][s'][e][b'] = tg[(a,e),(s',b')] / lam_{n-1}[a]; new
// Gamma_{n+1}[b'][t'][f][c] = tg[(b',t'),(f,c)] / lam_{n+1}[c].
// grid (blocks, items); side selects which site.
__global__ void k_store_gamma(const ChainDev* chains, const BondJob* jobs, int side) {
  const BondJob& J = jobs[blockIdx.y];
  const ChainDev& C = chains[J.chain];
  const int* D = J.dims;
  const int chi = D[D_CHI];
  if (side == 0) {
    const int a = D[D_A], e = D[D_E];
    double2* out = gamma_next(C, J.bond);
    const double* lam_l = C.lam + (long long)J.bond * C.chi_cap;
    const long long tot = (long long)a * e * 4 * chi;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
         idx += (long long)gridDim.x * blockDim.x) {
      // idx over output layout [a][s][e][b']
      const int bp = (int)(idx % chi);
      long long rest = idx / chi;
      const int ei = (int)(rest % e);
      rest /= e;
      const int s = (int)(rest % 4);
      const int ai = (int)(rest / 4);
      const double2 v = J.tg[(long long)(ai * e + ei) * (4 * chi) + s * chi + bp];
      out[idx] = cscale<double>(v, 1.0 / lam_l[ai]);
    }
  } else {
    const int f = D[D_F], c = D[D_C];
    double2* out = gamma_next(C, J.bond + 1);
    const double* lam_r = C.lam + (long long)(J.bond + 2) * C.chi_cap;
    const long long tot = (long long)chi * 4 * f * c;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
         idx += (long long)gridDim.x * blockDim.x)
      out[idx] = cscale<double>(J.tg[idx], 1.0 / lam_r[(int)(idx % c)]);
  }
}

// ------------------------------------------------------------- finalize
// one block per item
__global__ void k_finalize(const ChainDev* chains, const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.x];
  const ChainDev& C = chains[J.chain];
  const int chi = J.dims[D_CHI];
  __shared__ double red[4];
  double part = 0.0;
  for (int i = threadIdx.x; i < chi; i += blockDim.x) part += fmax(J.wk[i], 0.0);
  const double nrm2 = block_sum(part, red);
  const double nrm = sqrt(nrm2);
  double* lam = C.lam + (long long)(J.bond + 1) * C.chi_cap;
  for (int i = threadIdx.x; i < chi; i += blockDim.x) lam[i] = sqrt(fmax(J.wk[i], 0.0)) / nrm;
  if (threadIdx.x == 0) {
    const int* D = J.dims;
    int bad = 0;
    if (!(nrm > 0.0)) bad |= ST_ZERO;
    if (!isfinite(nrm) || !isfinite(J.norms[0])) bad |= ST_NONFINITE;
    if (chi < 1 || D[D_L] < 1 || D[D_R] < 1) bad |= ST_ZERO;
    if (bad) atomicOr(C.status, bad);
    else atomicAdd(C.log_scale, log(nrm));
    C.chi[J.bond + 1] = chi;
    C.parity[J.bond] ^= 1;
    C.parity[J.bond + 1] ^= 1;
  }
}

}  // namespace ptt
