// Chain-level kernels of PT-TEBD: PT-MPO absorption (Appendix A.2 (i)-(j)),
// left super-operator insertion for correlations (Appendix A.4) and the
// observable read-out through cap tensors (Appendix A.3, (k)-(l)).
#pragma once

#include "bond_kernels.h"

namespace ptt {

struct BathDev {
  int site, n_steps, diagonal, pad;
  const double2* tens;        // concatenated P_k
  const long long* toff;      // [n_steps] offsets of P_k
  const int* dims;            // [n_steps + 1]
  const double2* caps;        // concatenated c^(k)
  const long long* coff;      // [n_steps + 1]
};

// Gamma_n[a,s,e',b] = sum_e P_k[e,e',s] Gamma_n[a,s,e,b]            (diagonal)
//                   = sum_{e,s_in} P_k[e,e',s,s_in] Gamma_n[a,s_in,e,b] (dense)
// for one bath of one chain, by the blocks of the x dimension.  `k` is the
// 1-based step index.
__device__ inline void pt_absorb_one(const ChainDev& C, const BathDev& B, int k) {
  const int site = B.site;
  if (k < 1 || k > B.n_steps) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(C.status, ST_RANGE);
    return;
  }
  const int xin = B.dims[k - 1], xout = B.dims[k];
  const int a = C.chi[site], b = C.chi[site + 1], e = C.xi[site];
  if (e != xin) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(C.status, ST_RANGE);
    return;
  }
  const double2* P = B.tens + B.toff[k - 1];
  const double2* g = gamma_cur(C, site);
  double2* out = gamma_next(C, site);
  const long long tot = (long long)a * 4 * xout * b;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int bi = (int)(idx % b);
    long long rest = idx / b;
    const int ep = (int)(rest % xout);
    rest /= xout;
    const int s = (int)(rest % 4);
    const int ai = (int)(rest / 4);
    double2 acc = mk<double>(0.0, 0.0);
    if (B.diagonal) {
      for (int ei = 0; ei < e; ++ei)
        cfma<double>(acc, P[((long long)ei * xout + ep) * 4 + s], g[((long long)(ai * 4 + s) * e + ei) * b + bi]);
    } else {
      for (int ei = 0; ei < e; ++ei)
        for (int si = 0; si < 4; ++si)
          cfma<double>(acc, P[(((long long)ei * xout + ep) * 4 + s) * 4 + si],
                       g[((long long)(ai * 4 + si) * e + ei) * b + bi]);
    }
    out[idx] = acc;
  }
}

// grid (blocks, n_baths) on one chain
__global__ void k_pt_absorb(const ChainDev* chain, const BathDev* baths, int k) {
  pt_absorb_one(*chain, baths[blockIdx.y], k);
}

// after the absorption: new augmented dim and buffer swap of one bath site
__device__ inline void pt_commit_one(const ChainDev& C, const BathDev& B, int k) {
  if (k < 1 || k > B.n_steps || C.xi[B.site] != B.dims[k - 1]) return;
  C.xi[B.site] = B.dims[k];
  C.parity[B.site] ^= 1;
}

// grid 1, threads >= n_baths
__global__ void k_pt_commit(const ChainDev* chain, const BathDev* baths, int n_baths, int k) {
  const int i = threadIdx.x;
  if (i >= n_baths) return;
  pt_commit_one(*chain, baths[i], k);
}

// Batched form over many chains: one work item per (chain, bath); the step
// index of chain c is kstep[c] + 1, read on the device, so the launch is the
// same at every step (a captured graph replays it).
struct BathRef {
  int chain, pad;
  const BathDev* bath;
};

// grid (blocks, n_refs)
__global__ void k_pt_absorb_batch(const ChainDev* chains, const BathRef* refs, const int* kstep) {
  const BathRef& R = refs[blockIdx.y];
  pt_absorb_one(chains[R.chain], *R.bath, kstep[R.chain] + 1);
}

// one thread per reference
__global__ void k_pt_commit_batch(const ChainDev* chains, const BathRef* refs, int n_refs, const int* kstep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_refs) return;
  const BathRef& R = refs[i];
  pt_commit_one(chains[R.chain], *R.bath, kstep[R.chain] + 1);
}

// end of a batched step: every chain's step counter advances
__global__ void k_advance_steps(int* kstep, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) kstep[i] += 1;
}

// Gamma_i[a,s,e,b] <- sum_{s''} op[s,s''] Gamma_i[a,s'',e,b] (in place; one
// thread per (a,e,b) column).  op is a 4 x 4 Liouville-space super-operator.
__global__ void k_apply_site_op(const ChainDev* chain, int site, const double2* op) {
  const ChainDev& C = *chain;
  const int a = C.chi[site], e = C.xi[site], b = C.chi[site + 1];
  double2* g = gamma_cur(C, site);
  const long long tot = (long long)a * e * b;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int bi = (int)(idx % b);
    long long rest = idx / b;
    const int ei = (int)(rest % e);
    const int ai = (int)(rest / e);
    double2 in[4];
    for (int s = 0; s < 4; ++s) in[s] = g[((long long)(ai * 4 + s) * e + ei) * b + bi];
    for (int s = 0; s < 4; ++s) {
      double2 acc = mk<double>(0.0, 0.0);
      for (int q = 0; q < 4; ++q) cfma<double>(acc, op[s * 4 + q], in[q]);
      g[((long long)(ai * 4 + s) * e + ei) * b + bi] = acc;
    }
  }
}

// ------------------------------------------------------------- read-out
struct ObsScratch {
  double2* hat;       // [n_sites][chi_cap][4][chi_cap]  Gamma-hat with the cap contracted
  double2* lvec;      // [(n_sites + 1)][chi_cap] normalised left vectors
  double2* rvec;      // [(n_sites + 1)][chi_cap] normalised right vectors
  double* llog;       // [n_sites + 1] log of the left normalisations
  double* rlog;       // [n_sites + 1]
};

// Gamma-hat_n[a,s,b] = sum_e Gamma_n[a,s,e,b] c_n[e]; grid (blocks, n_sites)
__global__ void k_obs_hat(const ChainDev* chain, const BathDev* baths, const int* bath_of_site,
                          int step, ObsScratch S) {
  const ChainDev& C = *chain;
  const int site = blockIdx.y;
  const int a = C.chi[site], e = C.xi[site], b = C.chi[site + 1];
  const int bi_bath = bath_of_site[site];
  const double2* cap = nullptr;
  if (bi_bath >= 0) {
    const BathDev& B = baths[bi_bath];
    if (step >= 0 && step <= B.n_steps && B.dims[step] == e) cap = B.caps + B.coff[step];
    else if (e != 1) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(C.status, ST_RANGE);
      return;
    }
  }
  const double2* g = gamma_cur(C, site);
  double2* hat = S.hat + (long long)site * C.chi_cap * 4 * C.chi_cap;
  const long long tot = (long long)a * 4 * b;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int bi = (int)(idx % b);
    const long long as = idx / b;
    double2 acc = mk<double>(0.0, 0.0);
    for (int ei = 0; ei < e; ++ei) {
      const double2 gv = g[(as * e + ei) * b + bi];
      if (cap) cfma<double>(acc, cap[ei], gv);
      else acc = cadd<double>(acc, gv);
    }
    hat[idx] = acc;
  }
}

// Left and right trace-vector scans with normalisation (one block).
//   L_0 = [1],  L_{n+1}[b] = sum_a L_n[a] lam_n[a] T_n[a,b]
//   R_N = [1],  R_n[a]     = sum_b T_n[a,b] lam_{n+1}[b] R_{n+1}[b]
// with T_n[a,b] = sum_s t[s] hat_n[a,s,b], t = vec(identity).
__global__ void k_obs_scan(const ChainDev* chain, ObsScratch S) {
  const ChainDev& C = *chain;
  const int N = C.n_sites, cc = C.chi_cap;
  __shared__ double red[4];
  __shared__ double2 tmp[1024];
  if (threadIdx.x == 0) {
    S.lvec[0] = mk<double>(1.0, 0.0);
    S.llog[0] = 0.0;
    S.rvec[(long long)N * cc] = mk<double>(1.0, 0.0);
    S.rlog[N] = 0.0;
  }
  __syncthreads();
  for (int n = 0; n < N; ++n) {
    const int a = C.chi[n], b = C.chi[n + 1];
    const double* lam = C.lam + (long long)n * cc;
    const double2* hat = S.hat + (long long)n * cc * 4 * cc;
    const double2* lin = S.lvec + (long long)n * cc;
    double part = 0.0;
    for (int bi = threadIdx.x; bi < b; bi += blockDim.x) {
      double2 acc = mk<double>(0.0, 0.0);
      for (int ai = 0; ai < a; ++ai) {
        const double2 t = cadd<double>(hat[((long long)ai * 4 + 0) * b + bi], hat[((long long)ai * 4 + 3) * b + bi]);
        cfma<double>(acc, cscale<double>(lin[ai], lam[ai]), t);
      }
      tmp[bi] = acc;
      part = fmax(part, fmax(fabs(acc.x), fabs(acc.y)));
    }
    // max-abs normalisation
    __syncthreads();
    double mx = part;
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    double nrm = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) nrm = fmax(nrm, red[w]);
    if (!(nrm > 0.0)) nrm = 1.0;
    for (int bi = threadIdx.x; bi < b; bi += blockDim.x) S.lvec[(long long)(n + 1) * cc + bi] = cscale<double>(tmp[bi], 1.0 / nrm);
    if (threadIdx.x == 0) S.llog[n + 1] = S.llog[n] + log(nrm);
    __syncthreads();
  }
  for (int n = N - 1; n >= 0; --n) {
    const int a = C.chi[n], b = C.chi[n + 1];
    const double* lamr = C.lam + (long long)(n + 1) * cc;
    const double2* hat = S.hat + (long long)n * cc * 4 * cc;
    const double2* rin = S.rvec + (long long)(n + 1) * cc;
    double part = 0.0;
    for (int ai = threadIdx.x; ai < a; ai += blockDim.x) {
      double2 acc = mk<double>(0.0, 0.0);
      for (int bi = 0; bi < b; ++bi) {
        const double2 t = cadd<double>(hat[((long long)ai * 4 + 0) * b + bi], hat[((long long)ai * 4 + 3) * b + bi]);
        cfma<double>(acc, t, cscale<double>(rin[bi], lamr[bi]));
      }
      tmp[ai] = acc;
      part = fmax(part, fmax(fabs(acc.x), fabs(acc.y)));
    }
    __syncthreads();
    double mx = part;
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    double nrm = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) nrm = fmax(nrm, red[w]);
    if (!(nrm > 0.0)) nrm = 1.0;
    for (int ai = threadIdx.x; ai < a; ai += blockDim.x) S.rvec[(long long)n * cc + ai] = cscale<double>(tmp[ai], 1.0 / nrm);
    if (threadIdx.x == 0) S.rlog[n] = S.rlog[n + 1] + log(nrm);
    __syncthreads();
  }
}

// For each requested (site, o): out[i] = (num, den) with
//   num = L~_n lam_n O_n lam_{n+1} R~_{n+1},  O_n[a,b] = sum_s o[s] hat_n[a,s,b]
//   den = the same with o = t (the trace vector)
// so <O> = num / den; out also carries the log scale of the pair.
// grid n_ops, one block each.
__global__ void k_obs_ops(const ChainDev* chain, ObsScratch S, const int* sites, const double2* ovec,
                          double2* out, double* out_log) {
  const ChainDev& C = *chain;
  const int cc = C.chi_cap;
  const int i = blockIdx.x;
  const int n = sites[i];
  const int a = C.chi[n], b = C.chi[n + 1];
  const double* laml = C.lam + (long long)n * cc;
  const double* lamr = C.lam + (long long)(n + 1) * cc;
  const double2* hat = S.hat + (long long)n * cc * 4 * cc;
  const double2* lin = S.lvec + (long long)n * cc;
  const double2* rin = S.rvec + (long long)(n + 1) * cc;
  const double2* o = ovec + 4 * i;
  __shared__ double red[4];
  double2 num = mk<double>(0.0, 0.0), den = mk<double>(0.0, 0.0);
  for (long long idx = threadIdx.x; idx < (long long)a * b; idx += blockDim.x) {
    const int ai = (int)(idx / b), bi = (int)(idx - (long long)ai * b);
    const double2 w = cmul<double>(cscale<double>(lin[ai], laml[ai]), cscale<double>(rin[bi], lamr[bi]));
    double2 ov = mk<double>(0.0, 0.0);
    for (int s = 0; s < 4; ++s) cfma<double>(ov, o[s], hat[((long long)ai * 4 + s) * b + bi]);
    const double2 tv = cadd<double>(hat[((long long)ai * 4 + 0) * b + bi], hat[((long long)ai * 4 + 3) * b + bi]);
    cfma<double>(num, w, ov);
    cfma<double>(den, w, tv);
  }
  const double nr = block_sum(num.x, red), ni = block_sum(num.y, red);
  const double dr = block_sum(den.x, red), di = block_sum(den.y, red);
  if (threadIdx.x == 0) {
    out[2 * i] = mk<double>(nr, ni);
    out[2 * i + 1] = mk<double>(dr, di);
    out_log[i] = S.llog[n] + S.rlog[n + 1] + *C.log_scale;
  }
}

// Fluctuation and dissipation spectra (Sec. III.A) of a stationary
// auto-correlation C(tau_j) = <A(tau_j) A(0)>, tau_j = j dt, j = 0..n, of a
// Hermitian A, continued to negative times by C(-tau) = C(tau)^*.  With the
// trapezoid rule on [-n dt, n dt]:
//   S(w)   = dt sum_j c_j Re C(tau_j) cos(w tau_j)      (Fourier transform of 1/2 <{A(tau), A}>)
//   chi(w) = -dt sum_j c_j Im C(tau_j) sin(w tau_j)      (imaginary part of the transformed
//                                                         i Theta(tau) <[A(tau), A]>)
// where the sums run over j = 0..n, c_0 = 1, c_j = 2 for 0 < j < n, c_n = 1
// (the two halves of the symmetric interval folded onto j >= 0).  One
// thread per frequency; the sum over j in a fixed order.
__global__ void k_fdt_spectra(const double2* corr, int n, double dt, const double* omega, int n_omega, double* s_out,
                              double* chi_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_omega) return;
  const double w = omega[k];
  double s = 0.0, c = 0.0;
  for (int j = 0; j <= n; ++j) {
    const double cj = (j == 0 || j == n) ? 1.0 : 2.0;
    double sn, cs;
    sincos(w * j * dt, &sn, &cs);
    s += cj * corr[j].x * cs;
    c -= cj * corr[j].y * sn;
  }
  if (n == 0) c = 0.0;
  s_out[k] = dt * s;
  chi_out[k] = dt * c;
}

}  // namespace ptt
