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
//   heev      all eigenpairs of each Gram matrix
//   prod      B_L V_L (or U_L^H B_L), U_R^H B_R (or B_R V_R): the singular
//             values are the column (row) norms of these products, which
//             resolves them to working precision relative to themselves
//             (the square roots of Gram eigenvalues would only resolve them
//             to ~1e-8 of the largest); the eps rule on them gives l, r (d)-(e)
//   xy        X = S_L V_L^H (l x (s,b)) times lam_n on b;  Y = U_R S_R
//   p, gate   P[(l,s),(t,r)] = sum_b X Y;  D = G applied on (s,t)       (e)-(f)
//   rf        randomised range finder for the leading singular subspace of D
//             (Gaussian sketch, power iteration, orthonormalisation by the
//             eigendecomposition of the basis Gram matrix), Rayleigh-Ritz on
//             Q^H D (singular values again as row norms of W^H Q^H D) with
//             the eps rule, the chi_max cap and the tie rule            (f)-(g)
//   rebuild   Gamma_n' = lam_{n-1}^-1 U_L U^D,  Gamma_{n+1}' = V^D^H V_R^H
//             lam_{n+1}^-1; where the eigenvectors sit on the far side of B
//             the same products are evaluated as B V S^-1 U^D (resp.
//             V^D^H S^-1 U^H B), which is the identical algebra  (g)-(h)
//   finalize  new bond vector S^D / ||S^D||_2, log-scale += log ||S^D||_2
#pragma once

#include "device_common.h"
#include "gemm.h"
#include "gemm_mfma.h"
#include "heev.h"
#include "refine.h"

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
  double* work;          // [4] model flops F_a1..F_a4 of the bond updates so far (see k_finalize)
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
  D_RF,                        // 1: randomised range finder active; 0: Q = identity (M <= sketch cap)
  D_FB,                        // Gram size handed to the eigenvalue form of a second orthonormalisation pass (0: none)
  D_GS0, D_K1, D_GS2, D_K2,    // deflation: sketch width at entry, level-1 rank, residual Gram size (0: none), level-2 rank
  D_G2S, D_FB2,                // level-2 second-pass Gram size, its eigenvalue-form size (0: none)
  D_COUNT
};

enum StatusBits : int { ST_NONFINITE = 1, ST_ZERO = 2, ST_EIG = 4, ST_RANGE = 8, ST_NOCONV = 16 };
// bits of the per-slot eigensolver word (HeevJob::status)
enum EigBits : int { EIG_NOCONV = 1, EIG_NONFINITE = 4, EIG_SIZE = 8 };

struct BondJob {
  int chain;               // index into the chain array passed to the kernels
  int bond;                // sites bond, bond+1
  const double2* gate;     // [16][16] site-major
  int chi_max;
  int k_cap;               // capacity of the sketch-side buffers (ld of omega, ya, yb, za, zb, gk, vk);
                           // D is factorised exactly (Q = I) when M <= k_cap
  int k_sketch;            // sketch width cap of the range finder (<= k_cap)
  double eps;
  double floor_rel;        // mixed-precision noise floor of the truncation (0 in double precision)
  unsigned long long seed;
  int nb_cap;              // capacity of B Gram sizes (4 chi_cap); ld of gl/gr/vl/vr
  int dn_cap;              // capacity of M, N (4 nb_cap)
  int ldr;                 // leading dim of pr (max(xi_cap chi_cap, nb_cap))
  int* dims;               // [D_COUNT]
  int* estat;              // [1] eigensolver status of this slot's current update (EigBits)
  double* norms;           // [8]: ||D||_F^2, ||Q^H D||_F^2, extra tail, log-scale term,
                           //      largest Gram eigenvalue of the basis being orthonormalised
  double2 *bl, *br, *gl, *gr, *vl, *vr, *x, *y, *p, *d;
  double *wl, *wr, *wk;
  double *sl, *sr, *sk;    // singular values (norms) for B_L, B_R, D
  double2 *pl, *pr;        // B_L V_L or U_L^H B_L;  U_R^H B_R or B_R V_R
  double2 *tpl, *tvl, *tpr, *tvr;  // refinement temporaries
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
    *J.estat = 0;
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
  GK_PROD_B,       // sub 0: pl = B_L V_L (side 0) | U_L^H B_L (side 1)
                   // sub 1: pr = U_R^H B_R (side 0) | B_R V_R (side 1)
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
  GK_RESID,        // p -= ya bm (p holds a copy of D) (M x N), only if K < min(M, N)
  GK_GRAM_BM,      // gk = bm bm^H                     (KQ x KQ)
  GK_C,            // vdh = vk^H bm                    (KQ x N) = S V^D^H
  GK_UD,           // ud = ya vk                       (M x CHI)
  GK_NEWL,         // tg = U_L ud' (U_L = pl S_L^-1 on side 0, vl on side 1)      (rl x 4 chi)
  GK_NEWR,         // tg = vdh' V_R^H (V_R^H = S_R^-1 pr on side 0, vr^H on side 1) (4 chi x cr)
  // deflated orthonormalisation of the range finder's bases.  Basis X
  // (rows R) with scratch S and T: Y side X = ya, S = za, T = yb, R = M; Z
  // side X = za, S = ya, T = zb, R = N.  The kind is GK_DF + 2 op + side.
  GK_DF,
};
enum DeflOp : int {
  DF_APPLY1 = 0,   // S = T vk                         (R x Kb, k = GS)     Kb = KQ | KZ
  DF_C,            // gk = S^H X                       (K1 x GS2, k = R)
  DF_R,            // X -= S gk                        (R x GS2, k = K1)
  DF_GRAM2,        // gk = X^H X                       (GS2 x GS2, k = R)
  DF_APPLY2,       // T = X vk                         (R x K2, k = GS2)
  DF_C2,           // gk = S^H T                       (K1 x K2, k = R)
  DF_R2,           // T -= S gk                        (R x K2, k = K1)
  DF_GRAM2B,       // gk = T^H T                       (G2S x G2S, k = R)
  DF_APPLY2B,      // S[:, K1:] = T vk                 (R x K2, k = G2S)
  DF_OPS
};

struct GemmArgs {
  const double2* A; int lda; bool ca;
  const double2* B; int ldb; bool cb;
  double2* C; int ldc;
  int m, n, k;
  double alpha;
  bool acc;
};

__device__ inline bool gemm_args(const BondJob& J, int kind, int sub, GemmArgs& g) {
  const int* D = J.dims;
  const int kc = J.k_cap, nb = J.nb_cap;
  g.alpha = 1.0;
  g.acc = false;
  auto set = [&](const double2* A, int lda, bool ca, const double2* B, int ldb, bool cb, double2* C, int ldc,
                 int m, int n, int k) {
    g.A = A; g.lda = lda; g.ca = ca; g.B = B; g.ldb = ldb; g.cb = cb; g.C = C; g.ldc = ldc;
    g.m = m; g.n = n; g.k = k;
  };
  // the sketch / orthonormalisation / power-iteration products run only
  // when the range finder is active
  if (kind >= GK_SKETCH && kind <= GK_D_Z && D[D_RF] == 0) return false;
  if (kind >= GK_DF) {
    if (D[D_RF] == 0) return false;
    const int op = (kind - GK_DF) >> 1, side = (kind - GK_DF) & 1;
    double2* X = side ? J.za : J.ya;
    double2* S = side ? J.ya : J.za;
    double2* T = side ? J.zb : J.yb;
    const int R = side ? D[D_N] : D[D_M], kb = side ? D[D_KZ] : D[D_KQ];
    const int k1 = D[D_K1], gs2 = D[D_GS2], k2 = D[D_K2];
    // level 2 runs only where level 1 dropped directions
    if (op > DF_APPLY1 && gs2 == 0) return false;
    switch (op) {
      case DF_APPLY1: set(T, kc, false, J.vk, kc, false, S, kc, R, kb, D[D_GS]); break;
      case DF_C: set(S, kc, true, X, kc, false, J.gk, kc, k1, gs2, R); break;
      case DF_R: set(S, kc, false, J.gk, kc, false, X, kc, R, gs2, k1); g.alpha = -1.0; g.acc = true; break;
      case DF_GRAM2: set(X, kc, true, X, kc, false, J.gk, kc, gs2, gs2, R); break;
      case DF_APPLY2: set(X, kc, false, J.vk, kc, false, T, kc, R, k2, gs2); break;
      case DF_C2: set(S, kc, true, T, kc, false, J.gk, kc, k1, k2, R); break;
      case DF_R2: set(S, kc, false, J.gk, kc, false, T, kc, R, k2, k1); g.alpha = -1.0; g.acc = true; break;
      case DF_GRAM2B: set(T, kc, true, T, kc, false, J.gk, kc, D[D_G2S], D[D_G2S], R); break;
      case DF_APPLY2B: set(T, kc, false, J.vk, kc, false, S + k1, kc, R, k2, D[D_G2S]); break;
      default: return false;
    }
    return true;
  }
  switch (kind) {
    case GK_GRAM_B:
      if (sub == 0) {
        const int rl = D[D_RL], cl = D[D_CL];
        if (D[D_SL] == 0) set(J.bl, cl, true, J.bl, cl, false, J.gl, nb, cl, cl, rl);
        else set(J.bl, cl, false, J.bl, cl, true, J.gl, nb, rl, rl, cl);
      } else {
        const int rr = D[D_RR], cr = D[D_CR];
        if (D[D_SR] == 0) set(J.br, cr, false, J.br, cr, true, J.gr, nb, rr, rr, cr);
        else set(J.br, cr, true, J.br, cr, false, J.gr, nb, cr, cr, rr);
      }
      return true;
    case GK_PROD_B:
      if (sub == 0) {
        const int rl = D[D_RL], cl = D[D_CL], n = D[D_NL];
        if (D[D_SL] == 0) set(J.bl, cl, false, J.vl, nb, false, J.pl, nb, rl, n, cl);   // rl x n
        else set(J.vl, nb, true, J.bl, cl, false, J.pl, nb, n, cl, rl);                 // n x cl
      } else {
        const int rr = D[D_RR], cr = D[D_CR], n = D[D_NR];
        if (D[D_SR] == 0) set(J.vr, nb, true, J.br, cr, false, J.pr, J.ldr, n, cr, rr); // n x cr
        else set(J.br, cr, false, J.vr, nb, false, J.pr, J.ldr, rr, n, cr);            // rr x n
      }
      return true;
    case GK_P:
      set(J.x, D[D_B], false, J.y, 4 * D[D_R], false, J.p, 4 * D[D_R], 4 * D[D_L], 4 * D[D_R], D[D_B]);
      return true;
    case GK_SKETCH:
      set(J.d, D[D_N], false, J.omega, kc, false, J.ya, kc, D[D_M], D[D_K], D[D_N]);
      return true;
    case GK_GRAM_YA:
      set(J.ya, kc, true, J.ya, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_M]);
      return true;
    case GK_APPLY_YA:
      set(J.ya, kc, false, J.vk, kc, false, J.yb, kc, D[D_M], D[D_KQ], D[D_GS]);
      return true;
    case GK_GRAM_YB:
      set(J.yb, kc, true, J.yb, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_M]);
      return true;
    case GK_APPLY_YB:
      set(J.yb, kc, false, J.vk, kc, false, J.ya, kc, D[D_M], D[D_KQ], D[D_GS]);
      return true;
    case GK_DH_Q:
      set(J.d, D[D_N], true, J.ya, kc, false, J.za, kc, D[D_N], D[D_KQ], D[D_M]);
      return true;
    case GK_GRAM_ZA:
      set(J.za, kc, true, J.za, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_N]);
      return true;
    case GK_APPLY_ZA:
      set(J.za, kc, false, J.vk, kc, false, J.zb, kc, D[D_N], D[D_KZ], D[D_GS]);
      return true;
    case GK_GRAM_ZB:
      set(J.zb, kc, true, J.zb, kc, false, J.gk, kc, D[D_GS], D[D_GS], D[D_N]);
      return true;
    case GK_APPLY_ZB:
      set(J.zb, kc, false, J.vk, kc, false, J.za, kc, D[D_N], D[D_KZ], D[D_GS]);
      return true;
    case GK_D_Z:
      set(J.d, D[D_N], false, J.za, kc, false, J.ya, kc, D[D_M], D[D_KZ], D[D_N]);
      return true;
    case GK_QH_D:
      set(J.ya, kc, true, J.d, D[D_N], false, J.bm, D[D_N], D[D_KQ], D[D_N], D[D_M]);
      return true;
    case GK_RESID:
      if (D[D_K] >= min(D[D_M], D[D_N])) return false;
      set(J.ya, kc, false, J.bm, D[D_N], false, J.p, D[D_N], D[D_M], D[D_N], D[D_KQ]);
      g.alpha = -1.0;
      g.acc = true;
      return true;
    case GK_GRAM_BM:
      set(J.bm, D[D_N], false, J.bm, D[D_N], true, J.gk, kc, D[D_KQ], D[D_KQ], D[D_N]);
      return true;
    case GK_C:
      set(J.vk, kc, true, J.bm, D[D_N], false, J.vdh, D[D_N], D[D_KQ], D[D_N], D[D_KQ]);
      return true;
    case GK_UD:
      set(J.ya, kc, false, J.vk, kc, false, J.ud, D[D_CHI], D[D_M], D[D_CHI], D[D_KQ]);
      return true;
    case GK_NEWL:
      if (D[D_SL] == 0)  // tg (rl x 4chi) = ((B_L V_L) S_L^-1)[:, :l] ud'  (pl rescaled)
        set(J.pl, nb, false, J.ud, 4 * D[D_CHI], false, J.tg, 4 * D[D_CHI], D[D_RL], 4 * D[D_CHI], D[D_L]);
      else               // tg = U_L[:, :l] ud'
        set(J.vl, nb, false, J.ud, 4 * D[D_CHI], false, J.tg, 4 * D[D_CHI], D[D_RL], 4 * D[D_CHI], D[D_L]);
      return true;
    case GK_NEWR:
      if (D[D_SR] == 0)  // tg (4chi x cr) = vdh' (S_R^-1 U_R^H B_R)[:r, :]  (pr rescaled)
        set(J.vdh, D[D_R], false, J.pr, J.ldr, false, J.tg, D[D_CR], 4 * D[D_CHI], D[D_CR], D[D_R]);
      else               // tg = vdh' V_R[:, :r]^H
        set(J.vdh, D[D_R], false, J.vr, nb, true, J.tg, D[D_CR], 4 * D[D_CHI], D[D_CR], D[D_R]);
      return true;
    default:
      return false;
  }
}

// grid (tiles_m, tiles_n, items * subs)
// flops (may be null): accumulates 8 m n k per product (complex MAC = 8 flops)
__global__ void __launch_bounds__(GEMM_THREADS) k_bond_gemm(const BondJob* jobs, int kind, int subs, double* flops) {
  __shared__ GemmSmem<double> sm;
  const int item = blockIdx.z / subs, sub = blockIdx.z - item * subs;
  GemmArgs g;
  if (!gemm_args(jobs[item], kind, sub, g)) return;
  if (g.m <= 0 || g.n <= 0) return;
  if (flops && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
    atomicAdd(flops, 8.0 * (double)g.m * g.n * g.k);
  gemm_tile<double>(g.A, g.lda, g.ca, g.B, g.ldb, g.cb, g.C, g.ldc, g.m, g.n, g.k,
                    mk<double>(g.alpha, 0.0), g.acc, blockIdx.x, blockIdx.y, sm);
}

// The same products on the matrix cores; CT = double for the FP64 path,
// float for the single-precision contractions of the mixed path.
template <typename CT>
__global__ void __launch_bounds__(GEMM_THREADS) k_bond_gemm_mfma(const BondJob* jobs, int kind, int subs,
                                                                 double* flops) {
  __shared__ MfmaSmem<CT> sm;
  const int item = blockIdx.z / subs, sub = blockIdx.z - item * subs;
  GemmArgs g;
  if (!gemm_args(jobs[item], kind, sub, g)) return;
  if (g.m <= 0 || g.n <= 0) return;
  if (flops && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
    atomicAdd(flops, 8.0 * (double)g.m * g.n * g.k);
  gemm_tile_mfma<CT>(g.A, g.lda, g.ca, g.B, g.ldb, g.cb, g.C, g.ldc, g.m, g.n, g.k,
                     mk<double>(g.alpha, 0.0), g.acc, blockIdx.x, blockIdx.y, sm);
}

// Products that the mixed-precision path runs in single precision: the
// contractions that form D (P = X Y), the range finder's products with D,
// and the rebuild of the site tensors.  Gram matrices, the projections
// whose norms are singular values, and everything after them stay double.
__host__ __device__ inline bool gemm_kind_single(int kind) {
  return kind == GK_P || kind == GK_SKETCH || kind == GK_DH_Q || kind == GK_D_Z || kind == GK_UD ||
         kind == GK_NEWL || kind == GK_NEWR;
}

// --------------------------------------------- singular values and rules
// Truncation rule of Appendix A.2 on singular values s[0..n) given in
// (eigenvalue) order: the smallest rank c whose discarded tail
// sqrt(extra + sum_{i >= c} s_i^2) is strictly below eps * max(s); exact
// zeros are never kept; rank >= 1; an optional cap comes second.  A run of
// neighbours within a relative gap of 1e-6 is kept or dropped whole: its
// split subspace is not determined by the matrix to better than
// u sigma_1 / gap (u the unit roundoff), so an eps cut inside a run moves
// to its end (the tail only shrinks) and a cap inside one to its start.
// Runs on one thread.
//
// floor_rel > 0 (mixed-precision form): the matrix was contracted in single
// precision, so its singular values below c u_32 ||X||_F are rounding
// noise; the threshold of the discarded tail is then
// max(eps sigma_max, floor_rel ||X||_F), ||X||_F^2 = extra + sum s_i^2.
// Without it the noise directions are kept, and lambda^-1 in the rebuild
// amplifies their single-precision errors into the site tensors.
constexpr double RUN_GAP = 1e-6;
__device__ inline int truncation_rank(const double* s, int n, double eps, double extra, int cap,
                                      double floor_rel = 0.0) {
  double smax = 0.0, tot = extra;
  int npos = 0;
  for (int i = 0; i < n; ++i) {
    smax = fmax(smax, s[i]);
    if (s[i] > 0.0) npos = i + 1;
    tot += s[i] * s[i];
  }
  if (npos == 0) return 0;
  const double thr = fmax(eps * smax, floor_rel * sqrt(tot));
  int keep = npos;
  double tail = extra;
  for (int i = npos - 1; i >= 1; --i) {
    tail += s[i] * s[i];
    if (sqrt(tail) < thr) keep = i;
    else break;
  }
  while (keep < npos && s[keep - 1] - s[keep] < RUN_GAP * s[keep - 1]) ++keep;
  if (cap > 0 && keep > cap) {
    keep = cap;
    while (keep > 1 && s[keep - 1] - s[keep] < RUN_GAP * s[keep - 1]) --keep;
  }
  return max(keep, 1);
}

// Truncation ranks l, r from the (refined) singular values of B_L, B_R:
// eps rule only.  One thread per item.
__global__ void k_rule_b(const BondJob* jobs, int n_items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const BondJob& J = jobs[i];
  int* D = J.dims;
  D[D_L] = truncation_rank(J.sl, D[D_NL], J.eps, 0.0, 0, J.floor_rel);
  D[D_R] = truncation_rank(J.sr, D[D_NR], J.eps, 0.0, 0, J.floor_rel);
  // D is formed from X / s_L,max and Y / s_R,max (unit scale whatever the
  // scale of the state, so single-precision products neither overflow nor
  // underflow); log(s_L,max s_R,max) goes to the log-scale with log ||S^D||
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < D[D_L]; ++k) sx = fmax(sx, J.sl[k]);
  for (int k = 0; k < D[D_R]; ++k) sy = fmax(sy, J.sr[k]);
  J.norms[5] = sx > 0.0 ? 1.0 / sx : 0.0;
  J.norms[6] = sy > 0.0 ? 1.0 / sy : 0.0;
  J.norms[7] = (sx > 0.0 && sy > 0.0) ? log(sx) + log(sy) : 0.0;
}

// ------------------------------------------------------ X, Y (elementwise)
// X (l x cl) times lam_n on the b index:  side 0: X[i,col] = s_i conj(V_L[col,i]);
// side 1: X = (U_L^H B_L)[:l].  Y (rr x r): side 0: Y[row,j] = U_R[row,j] s_j;
// side 1: Y = (B_R V_R)[:, :r].  grid (blocks, items)
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
      double2 v;
      if (D[D_SL] == 0) v = cscale<double>(cconj<double>(J.vl[(long long)col * nb + i]), J.sl[i]);
      else v = J.pl[(long long)i * nb + col];
      J.x[idx] = cscale<double>(v, lam_c[col % b] * J.norms[5]);
    } else {
      const long long j = idx - nx;
      const int row = (int)(j / r), k = (int)(j - (long long)row * r);
      const double2 v = (D[D_SR] == 0) ? cscale<double>(J.vr[(long long)row * nb + k], J.sr[k])
                                       : J.pr[(long long)row * J.ldr + k];
      J.y[j] = cscale<double>(v, J.norms[6]);
    }
  }
}

// ------------------------------------------------------------ gate on P
// D[(l,s'),(t',r)] = sum_{s,t} G[(s',t'),(s,t)] P[(l,s),(t,r)]; also sets
// M, N and the sketch width, accumulates ||D||_F^2.  grid (blocks, items)
template <typename CT>
__global__ void k_apply_gate(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  int* D = J.dims;
  const int l = D[D_L], r = D[D_R];
  const int M = 4 * l, N = 4 * r;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D[D_M] = M;
    D[D_N] = N;
    const int k = min(min(M, N), J.k_sketch);
    D[D_K] = k;
    // M <= k_cap: the identity is an orthonormal basis of the whole row
    // space of D, so no range finder is needed (exact)
    const int rf = (M > J.k_cap) ? 1 : 0;
    D[D_RF] = rf;
    D[D_GS] = rf ? k : 0;
    if (!rf) D[D_KQ] = M;
    // sizes read by launches that run for every item (0 = nothing to do);
    // the range-finder steps set them for their own items
    D[D_FB] = 0;
    D[D_GS0] = 0;
    D[D_K1] = 0;
    D[D_GS2] = 0;
    D[D_K2] = 0;
    D[D_G2S] = 0;
    D[D_FB2] = 0;
  }
  __shared__ cx<CT> g[256];
  __shared__ double red[4];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) g[i] = mk<CT>((CT)J.gate[i].x, (CT)J.gate[i].y);
  __syncthreads();
  double part = 0.0;
  const long long npairs = (long long)l * r;
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < npairs;
       pr += (long long)gridDim.x * blockDim.x) {
    const int li = (int)(pr / r), ri = (int)(pr - (long long)li * r);
    cx<CT> in[16];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 v = J.p[(long long)(li * 4 + s) * N + t * r + ri];
        in[s * 4 + t] = mk<CT>((CT)v.x, (CT)v.y);
      }
    // one output row of the gate at a time: unrolling all four hoists the
    // 256 gate entries out of LDS into registers and spills
#pragma unroll 1
    for (int so = 0; so < 4; ++so)
#pragma unroll
      for (int to = 0; to < 4; ++to) {
        cx<CT> acc = mk<CT>(0, 0);
#pragma unroll
        for (int q = 0; q < 16; ++q) cfma<CT>(acc, g[(so * 4 + to) * 16 + q], in[q]);
        const double2 o = mk<double>((double)acc.x, (double)acc.y);
        J.d[(long long)(li * 4 + so) * N + to * r + ri] = o;
        part += cabs2<double>(o);
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
  if (J.dims[D_RF] == 0) {  // Q = identity (M x M) in ya
    const int M = J.dims[D_M];
    const long long tot = (long long)M * M;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
         idx += (long long)gridDim.x * blockDim.x) {
      const int r = (int)(idx / M), c = (int)(idx - (long long)r * M);
      J.ya[(long long)r * J.k_cap + c] = mk<double>(r == c ? 1.0 : 0.0, 0.0);
    }
    return;
  }
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

// deflation bookkeeping, one thread per item (range finder jobs only).
// stage 0: before level 1 (GS0 = GS); stage 1: after the level-1 eigenvalue
// pass (largest Gram eigenvalue); stage 2: after level 1 (K1 = Kb, GS2 =
// GS0 if directions were dropped); stage 3: before the level-2 second pass
// (K2 <= GS0 - K1, G2S = K2); stage 4: after level 2 (Kb = K1 + K2).
__global__ void k_defl_dims(const BondJob* jobs, int n_items, int stage, int side) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const BondJob& J = jobs[i];
  int* D = J.dims;
  if (!D[D_RF]) return;
  const int kb = side ? D_KZ : D_KQ;
  switch (stage) {
    case 0: D[D_GS0] = D[D_GS]; D[D_GS2] = 0; D[D_K2] = 0; D[D_G2S] = 0; break;
    case 1: J.norms[4] = J.wk[0]; break;
    case 2: D[D_K1] = D[kb]; D[D_GS2] = (D[kb] < D[D_GS0]) ? D[D_GS0] : 0; D[D_K2] = 0; break;
    case 3:  // the two levels together span at most the sketch width
      if (D[D_GS2]) D[D_K2] = max(0, min(D[D_K2], D[D_GS0] - D[D_K1]));
      D[D_G2S] = D[D_GS2] ? D[D_K2] : 0;
      break;
    case 4: if (D[D_GS2]) D[kb] = D[D_K1] + D[D_K2]; break;
  }
}

// X = S (R x Kb) after a deflated orthonormalisation.  grid (blocks, items)
__global__ void k_defl_copy(const BondJob* jobs, int side) {
  const BondJob& J = jobs[blockIdx.y];
  const int* D = J.dims;
  if (!D[D_RF]) return;
  double2* X = side ? J.za : J.ya;
  const double2* S = side ? J.ya : J.za;
  const int R = side ? D[D_N] : D[D_M], kb = side ? D[D_KZ] : D[D_KQ];
  const long long tot = (long long)R * kb;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / kb), c = (int)(idx - (long long)r * kb);
    X[(long long)r * J.k_cap + c] = S[(long long)r * J.k_cap + c];
  }
}

// small dims bookkeeping kernel: dims[dst] = dims[src] for every item
// (only where the range finder is active if only_rf)
__global__ void k_copy_dim(const BondJob* jobs, int n_items, int dst, int src, int only_rf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_items && (!only_rf || jobs[i].dims[D_RF])) jobs[i].dims[dst] = jobs[i].dims[src];
}

// p = D (copy) when the sketch does not span D's whole range; the residual
// D - Q Q^H D is then formed by GK_RESID.  grid (blocks, items)
__global__ void k_resid_copy(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  const int* D = J.dims;
  const int M = D[D_M], N = D[D_N];
  if (D[D_K] >= min(M, N)) return;
  const long long tot = (long long)M * N;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x)
    J.p[idx] = J.d[idx];
}

// extra tail = ||D - Q Q^H D||_F^2 (0 when the sketch spans the range)
// -> norms[2].  One block per item.
// partial sums of |residual|^2, one per block, into wk[blockIdx.x] (the
// eigenvalue array is free between the orthonormalisations and the
// Rayleigh-Ritz step).  grid (RESID_BLOCKS, items)
constexpr int RESID_BLOCKS = 64;
__global__ void k_resid_partial(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  const int* D = J.dims;
  const int M = D[D_M], N = D[D_N];
  __shared__ double red[16];
  double part = 0.0;
  if (D[D_K] < min(M, N))
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (long long)M * N;
         idx += (long long)gridDim.x * blockDim.x)
      part += cabs2<double>(J.p[idx]);
  const double tot = block_sum(part, red);
  if (threadIdx.x == 0) J.wk[blockIdx.x] = tot;
}

// norms[2] = the partial sums added in block order.  One thread per item.
__global__ void k_resid_norm(const BondJob* jobs, int n_items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const BondJob& J = jobs[i];
  double tot = 0.0;
  for (int b = 0; b < RESID_BLOCKS; ++b) tot += J.wk[b];
  J.norms[2] = tot;
}

// New bond dimension from the (refined) singular values of D: eps rule with
// the energy outside the sketch as extra tail, chi_max cap, tie rule.
// One thread per item.
__global__ void k_rule_d(const BondJob* jobs, int n_items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const BondJob& J = jobs[i];
  int* D = J.dims;
  D[D_CHI] = truncation_rank(J.sk, D[D_KQ], J.eps, J.norms[2], J.chi_max, J.floor_rel);
}

// vdh rows /= s_i (V^D^H = S^-1 W^H B).  Side-0 rebuilds: the columns of
// pl = B_L V_L (norms s_L) and the rows of pr = U_R^H B_R (norms s_R) are
// divided by those norms, which turns them into U_L and V_R^H; the rebuild
// products then multiply factors of unit scale (safe in single precision).
__global__ void k_scale_factors(const BondJob* jobs) {
  const BondJob& J = jobs[blockIdx.y];
  const int* D = J.dims;
  const int chi = D[D_CHI], N = D[D_N], l = D[D_L], r = D[D_R];
  const long long nv = (long long)chi * N;
  const long long npl = (D[D_SL] == 0) ? (long long)D[D_RL] * l : 0;
  const long long npr = (D[D_SR] == 0) ? (long long)r * D[D_CR] : 0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nv + npl + npr;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < nv) {
      const int i = (int)(idx / N);
      J.vdh[idx] = cscale<double>(J.vdh[idx], 1.0 / fmax(J.sk[i], 1e-300));
    } else if (idx < nv + npl) {
      const long long j = idx - nv;
      const int row = (int)(j / l), c = (int)(j - (long long)row * l);
      double2* at = J.pl + (long long)row * J.nb_cap + c;
      *at = cscale<double>(*at, 1.0 / fmax(J.sl[c], 1e-300));
    } else {
      const long long j = idx - nv - npl;
      const int row = (int)(j / D[D_CR]), c = (int)(j - (long long)row * D[D_CR]);
      double2* at = J.pr + (long long)row * J.ldr + c;
      *at = cscale<double>(*at, 1.0 / fmax(J.sr[row], 1e-300));
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
  for (int i = threadIdx.x; i < chi; i += blockDim.x) part += J.sk[i] * J.sk[i];
  const double nrm = sqrt(block_sum(part, red));
  double* lam = C.lam + (long long)(J.bond + 1) * C.chi_cap;
  for (int i = threadIdx.x; i < chi; i += blockDim.x) lam[i] = J.sk[i] / nrm;
  if (threadIdx.x == 0) {
    const int* D = J.dims;
    int bad = 0;
    if (!(nrm > 0.0)) bad |= ST_ZERO;
    if (!isfinite(nrm) || !isfinite(J.norms[0])) bad |= ST_NONFINITE;
    if (chi < 1 || D[D_L] < 1 || D[D_R] < 1) bad |= ST_ZERO;
    // the eigensolver's word of this update goes to the chain being stepped
    const int es = *J.estat;
    if (es & EIG_NOCONV) bad |= ST_NOCONV;
    if (es & EIG_NONFINITE) bad |= ST_EIG;
    if (es & EIG_SIZE) bad |= ST_RANGE;
    if (bad) atomicOr(C.status, bad);
    J.norms[3] = bad ? 0.0 : log(nrm) + J.norms[7];   // summed in item order by k_logscale
    // minimal algorithmic work of this update from its dims (complex
    // multiply-add = 8 flops, d^2 = 4): rank-l / rank-r factorisations of
    // B_L, B_R (two passes each); the X lambda Y contraction and the 16 x 16
    // gate; the top-chi' part of D (two passes); the two rebuild products
    const double a = D[D_A], e = D[D_E], b = D[D_B], f = D[D_F], c = D[D_C];
    const double l = D[D_L], r = D[D_R], cp = chi;
    atomicAdd(C.work + 0, 16.0 * (a * e) * (4.0 * b) * l + 16.0 * (4.0 * b) * (f * c) * r);
    atomicAdd(C.work + 1, 8.0 * (4.0 * l) * b * (4.0 * r) + 8.0 * 256.0 * l * r);
    atomicAdd(C.work + 2, 16.0 * (4.0 * l) * (4.0 * r) * cp);
    atomicAdd(C.work + 3, 8.0 * (a * e) * l * (4.0 * cp) + 8.0 * (4.0 * cp) * r * (f * c));
    C.chi[J.bond + 1] = chi;
    C.parity[J.bond] ^= 1;
    C.parity[J.bond + 1] ^= 1;
  }
}

// log-scale += log ||S^D|| of every item, in item order (deterministic).
__global__ void k_logscale(const ChainDev* chains, const BondJob* jobs, int n_items) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i < n_items; ++i) *chains[jobs[i].chain].log_scale += jobs[i].norms[3];
}

}  // namespace ptt
