// PT-TEBD engine and C ABI (include/pt_tebd.h).
#include "pt_tebd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "chain_kernels.h"
#include "cholqr.h"
#include "host_math.h"
#include "tempo_kernels.h"

using ptt::BathDev;
using ptt::BondJob;
using ptt::ChainDev;
using ptt::cplx;
using ptt::HeevJob;
using ptt::ObsScratch;

namespace {

constexpr int kThreads = 256;

// ------------------------------------------------------------- bump alloc
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct Sublayer {
  std::vector<int> bonds;
  BondJob* jobs = nullptr;       // device
  HeevJob* heev_b = nullptr;     // device [2 n]
  HeevJob* heev_oy = nullptr;    // device [n]
  HeevJob* heev_oz = nullptr;    // device [n]
  HeevJob* heev_oyb = nullptr;   // device [n]: eigenvalue form of the second pass (size dims[D_FB])
  HeevJob* heev_ozb = nullptr;   // device [n]
  HeevJob* heev_l2 = nullptr;    // device [n]: deflation level 2 (size dims[D_GS2])
  HeevJob* heev_l2b = nullptr;   // device [n]: its second pass in eigenvalue form (size dims[D_FB2])
  HeevJob* heev_rr = nullptr;    // device [n]
  ptt::RefineJob* ref_b = nullptr;  // device [2 n]: B_L, B_R
  ptt::RefineJob* ref_d = nullptr;  // device [n]
  HeevJob* heev_ref_b = nullptr;    // device [2 n]
  HeevJob* heev_ref_d = nullptr;    // device [n]
  std::vector<BondJob> host_jobs;
};

struct Caps {
  int n_sites, chi_cap, xi_cap, nb, dn, kc, ks, nh, n_slots;
  long long gam_cap;
};

// What a sublayer's launch sequence needs besides its job tables: the
// stream, the capacities that size the grids (the largest over the chains
// of a batch) and the range finder's and refinement's settings.
struct Exec {
  hipStream_t stream;
  Caps cap;
  int power_iters;
  bool cholqr, deflate;
  int refine_levels;
  double refine_tau;
};

}  // namespace

struct pt_tebd {
  // configuration
  int n_sites = 0, d = 2;
  double dt = 0.0;
  int chi_max = 1, xi_max = 1;
  double eps = 0.0;
  pt_tebd_precision precision = PT_TEBD_FP64;
  unsigned long long seed = 0;
  int power_iters = 2;
  bool cholqr = true;      // second orthonormalisation pass by Cholesky QR
  bool deflate = true;     // two-level (deflated) orthonormalisation of the range finder's bases
  int oversample = 64;
  int refine_levels = 0;   // block refinement levels (PT_TEBD_REFINE_LEVELS)
  int gemm_valu = 0;       // measurement switch PT_TEBD_GEMM_VALU: the VALU tile for every product
  unsigned mixed_mask = ~(1u << 30);  // measurement switch PT_TEBD_MIXED_KINDS: bit k = product kind k runs single
  double refine_tau = 1e-4;
  int pt_steps = 0;           // shortest PT-MPO length
  Caps cap{};
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<std::vector<cplx>> gates_host;
  // device
  ChainDev* chains = nullptr;  // [2]: main, fork
  ChainDev chain_host[2];
  double2* gates = nullptr;
  BathDev* baths = nullptr;
  int n_baths = 0;
  int* bath_of_site = nullptr;
  std::vector<int> bath_of_site_host;
  ObsScratch obs{};
  int ops_cap = 0;
  int* ops_sites = nullptr;
  double2* ops_vec = nullptr;
  double2* ops_out = nullptr;
  double* ops_log = nullptr;
  double2* site_op = nullptr;  // [16] super-operator for correlate
  Sublayer sub_even, sub_odd;  // 1-based even bonds (0-based odd), 1-based odd bonds
  int step = 0;
  std::string err;
  // per-launch timing of one kernel class (measurement support)
  int timing_class = 0;
  std::vector<hipEvent_t> events;  // start/end pairs, reused
  size_t events_used = 0;
  double* timing_flops = nullptr;  // device accumulator of algorithmic flops
};

namespace {

int env_int(const char* name, int dflt);

Caps compute_caps(const pt_tebd_config* cfg, int oversample) {
  Caps c{};
  c.n_sites = cfg->n_sites;
  c.chi_cap = std::max(1, cfg->chi_max);
  c.xi_cap = std::max(1, cfg->xi_max);
  c.nb = 4 * c.chi_cap;
  c.dn = 4 * c.nb;
  // the eigensolver holds one problem of size <= 1024 per workgroup.  The
  // range finder sketches chi_max + oversample columns; D with at most
  // max(that, 4 chi_max) rows is factorised exactly instead (the Gram
  // matrix of D is then no larger than those of B_L and B_R)
  c.ks = std::min({c.dn, c.chi_cap + oversample, 1024});
  c.kc = std::max(c.ks, std::min({c.dn, env_int("PT_TEBD_EXACT_ROWS", c.nb), 1024}));
  c.nh = std::max(c.nb, c.kc);
  c.n_slots = cfg->n_sites / 2;  // max(#even, #odd) bonds = floor(N/2)
  c.gam_cap = (long long)c.chi_cap * 4 * c.xi_cap * c.chi_cap;
  return c;
}

struct DevPtrs {
  // per chain (x2)
  double2* gam[2];
  int* parity[2];
  int* chi[2];
  int* xi[2];
  double* lam[2];
  double* log_scale[2];
  int* status[2];
  double* work[2];
  ChainDev* chains;
  double2* gates;
  BathDev* baths;
  int* bath_of_site;
  std::vector<double2*> bath_tens;
  std::vector<long long*> bath_toff;
  std::vector<int*> bath_dims;
  std::vector<double2*> bath_caps;
  std::vector<long long*> bath_coff;
  ObsScratch obs;
  int* ops_sites;
  double2* ops_vec;
  double2* ops_out;
  double* ops_log;
  double2* site_op;
  double* timing_flops;
  std::vector<BondJob> slots;          // scratch per slot (bond fields unset)
  std::vector<double2*> h_refl[2];
  std::vector<double*> h_tri[2], h_work[2], h_z[2];
  BondJob* jobs[2];
  HeevJob *hb[2], *hoy[2], *hoz[2], *hoyb[2], *hozb[2], *hl2[2], *hl2b[2], *hrr[2], *hrb[2], *hrd[2];
  ptt::RefineJob *rb[2], *rd[2];
  std::vector<int*> blk;   // per slot: 3 x [2]
};

// Walk the workspace layout once with a null base (sizes only) or with the
// real base (pointers).
size_t layout(const Caps& c, const pt_tebd_config* cfg, const std::vector<long long>& bath_tens_len,
              const std::vector<long long>& bath_caps_len, void* base, DevPtrs* out) {
  Bump bp(base);
  DevPtrs P;
  const int N = c.n_sites;
  for (int k = 0; k < 2; ++k) {
    P.gam[k] = bp.take<double2>((size_t)N * 2 * c.gam_cap);
    P.parity[k] = bp.take<int>(N);
    P.chi[k] = bp.take<int>(N + 1);
    P.xi[k] = bp.take<int>(N);
    P.lam[k] = bp.take<double>((size_t)(N + 1) * c.chi_cap);
    P.log_scale[k] = bp.take<double>(1);
    P.status[k] = bp.take<int>(1);
    P.work[k] = bp.take<double>(4);
  }
  P.chains = bp.take<ChainDev>(2);
  P.timing_flops = bp.take<double>(4);
  P.gates = bp.take<double2>((size_t)std::max(N - 1, 1) * 256);
  const int nbath = cfg->n_baths;
  P.baths = bp.take<BathDev>(std::max(nbath, 1));
  P.bath_of_site = bp.take<int>(N);
  for (int i = 0; i < nbath; ++i) {
    const int m = cfg->baths[i].n_steps;
    P.bath_tens.push_back(bp.take<double2>(bath_tens_len[i]));
    P.bath_toff.push_back(bp.take<long long>(m));
    P.bath_dims.push_back(bp.take<int>(m + 1));
    P.bath_caps.push_back(bp.take<double2>(bath_caps_len[i]));
    P.bath_coff.push_back(bp.take<long long>(m + 1));
  }
  P.obs.hat = bp.take<double2>((size_t)N * c.chi_cap * 4 * c.chi_cap);
  P.obs.lvec = bp.take<double2>((size_t)(N + 1) * c.chi_cap);
  P.obs.rvec = bp.take<double2>((size_t)(N + 1) * c.chi_cap);
  P.obs.llog = bp.take<double>(N + 1);
  P.obs.rlog = bp.take<double>(N + 1);
  const int ops_cap = 8 * N + 8;
  P.ops_sites = bp.take<int>(ops_cap);
  P.ops_vec = bp.take<double2>((size_t)ops_cap * 4);
  P.ops_out = bp.take<double2>((size_t)ops_cap * 2);
  P.ops_log = bp.take<double>(ops_cap);
  P.site_op = bp.take<double2>(16);
  const size_t rl = (size_t)c.chi_cap * c.xi_cap, nb = c.nb, dn = c.dn, kc = c.kc, nh = c.nh;
  for (int s = 0; s < c.n_slots; ++s) {
    BondJob J{};
    J.dims = bp.take<int>(ptt::D_COUNT);
    J.estat = bp.take<int>(1);
    J.norms = bp.take<double>(8);
    J.bl = bp.take<double2>(rl * nb);
    J.br = bp.take<double2>(nb * rl);
    J.gl = bp.take<double2>(nb * nb);
    J.gr = bp.take<double2>(nb * nb);
    J.vl = bp.take<double2>(nb * nb);
    J.vr = bp.take<double2>(nb * nb);
    J.wl = bp.take<double>(nh);
    J.wr = bp.take<double>(nh);
    J.x = bp.take<double2>(nb * nb);
    J.y = bp.take<double2>(nb * nb);
    J.p = bp.take<double2>(dn * dn);
    J.d = bp.take<double2>(dn * dn);
    J.wk = bp.take<double>(nh);
    J.sl = bp.take<double>(nh);
    J.sr = bp.take<double>(nh);
    J.sk = bp.take<double>(nh);
    J.pl = bp.take<double2>(std::max(rl, nb) * nb);
    J.pr = bp.take<double2>(nb * std::max(rl, nb));
    J.tpl = bp.take<double2>(std::max(rl, nb) * nb);
    J.tvl = bp.take<double2>(nb * nb);
    J.tpr = bp.take<double2>(nb * std::max(rl, nb));
    J.tvr = bp.take<double2>(nb * nb);
    P.blk.push_back(bp.take<int>(6));
    J.omega = bp.take<double2>(dn * kc);
    J.ya = bp.take<double2>(dn * kc);
    J.yb = bp.take<double2>(dn * kc);
    J.za = bp.take<double2>(dn * kc);
    J.zb = bp.take<double2>(dn * kc);
    J.gk = bp.take<double2>(kc * kc);
    J.vk = bp.take<double2>(kc * kc);
    J.bm = bp.take<double2>(kc * dn);
    J.ud = bp.take<double2>(dn * c.chi_cap);
    J.vdh = bp.take<double2>(kc * dn);
    J.t1 = nullptr;
    J.tg = bp.take<double2>(4 * (size_t)c.chi_cap * rl);
    P.slots.push_back(J);
    for (int set = 0; set < 2; ++set) {
      P.h_refl[set].push_back(bp.take<double2>(nh * nh));
      P.h_tri[set].push_back(bp.take<double>(6 * nh));
      P.h_work[set].push_back(bp.take<double>(8 * nh * nh));
      P.h_z[set].push_back(bp.take<double>(nh * nh));
    }
  }
  for (int par = 0; par < 2; ++par) {
    const int n = std::max(c.n_slots, 1);
    P.jobs[par] = bp.take<BondJob>(n);
    P.hb[par] = bp.take<HeevJob>(2 * n);
    P.hoy[par] = bp.take<HeevJob>(n);
    P.hoz[par] = bp.take<HeevJob>(n);
    P.hoyb[par] = bp.take<HeevJob>(n);
    P.hozb[par] = bp.take<HeevJob>(n);
    P.hl2[par] = bp.take<HeevJob>(n);
    P.hl2b[par] = bp.take<HeevJob>(n);
    P.hrr[par] = bp.take<HeevJob>(n);
    P.hrb[par] = bp.take<HeevJob>(2 * n);
    P.hrd[par] = bp.take<HeevJob>(n);
    P.rb[par] = bp.take<ptt::RefineJob>(2 * n);
    P.rd[par] = bp.take<ptt::RefineJob>(n);
  }
  if (out) *out = P;
  return bp.off + 256;
}

bool check(hipError_t e, pt_tebd* h, const char* what) {
  if (e == hipSuccess) return true;
  if (h) h->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

pt_tebd_status validate(const pt_tebd_config* cfg, std::string& err) {
  if (!cfg) { err = "null config"; return PT_TEBD_EINVAL; }
  if (cfg->n_sites < 1) { err = "n_sites must be >= 1"; return PT_TEBD_EINVAL; }
  if (cfg->d != 2) { err = "only d = 2 (spin-1/2) sites are supported"; return PT_TEBD_EINVAL; }
  if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) { err = "dt must be positive"; return PT_TEBD_EINVAL; }
  if (cfg->chi_max < 1 || cfg->chi_max > 256) { err = "chi_max must be in [1, 256]"; return PT_TEBD_EINVAL; }
  if (cfg->xi_max < 1 || cfg->xi_max > 1024) { err = "xi_max must be in [1, 1024]"; return PT_TEBD_EINVAL; }
  if (!(cfg->svd_rel_cutoff >= 0.0) || !(cfg->svd_rel_cutoff < 1.0)) { err = "svd_rel_cutoff must be in [0, 1)"; return PT_TEBD_EINVAL; }
  if (!cfg->h_site || !cfg->rho0 || (cfg->n_sites > 1 && !cfg->h_bond)) { err = "missing h_site, h_bond or rho0"; return PT_TEBD_EINVAL; }
  if (cfg->n_lindblad < 0 || (cfg->n_lindblad > 0 && !cfg->lindblad)) { err = "bad lindblad"; return PT_TEBD_EINVAL; }
  if (cfg->precision != PT_TEBD_FP64 && cfg->precision != PT_TEBD_FP32_MIXED) { err = "bad precision"; return PT_TEBD_EINVAL; }
  if (cfg->n_baths < 0 || cfg->n_baths > cfg->n_sites || (cfg->n_baths > 0 && !cfg->baths)) { err = "bad baths"; return PT_TEBD_EINVAL; }
  const int N = cfg->n_sites;
  auto herm = [](const double* m, int n) {
    double scale = 0.0, dev = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double ar = m[2 * (i * n + j)], ai = m[2 * (i * n + j) + 1];
        const double br = m[2 * (j * n + i)], bi = -m[2 * (j * n + i) + 1];
        if (!std::isfinite(ar) || !std::isfinite(ai)) return false;
        scale = std::max(scale, std::fabs(ar) + std::fabs(ai));
        dev = std::max(dev, std::fabs(ar - br) + std::fabs(ai - bi));
      }
    return dev <= 1e-10 * std::max(scale, 1.0);
  };
  for (int n = 0; n < N; ++n)
    if (!herm(cfg->h_site + 8 * n, 2)) { err = "h_site must be finite and Hermitian"; return PT_TEBD_EINVAL; }
  for (int b = 0; b + 1 < N; ++b)
    if (!herm(cfg->h_bond + 32 * b, 4)) { err = "h_bond must be finite and Hermitian"; return PT_TEBD_EINVAL; }
  for (int i = 0; i < 8 * N; ++i)
    if (!std::isfinite(cfg->rho0[i])) { err = "rho0 must be finite"; return PT_TEBD_EINVAL; }
  std::vector<int> used(N, 0);
  for (int i = 0; i < cfg->n_baths; ++i) {
    const pt_tebd_bath& b = cfg->baths[i];
    if (b.site < 0 || b.site >= N || used[b.site]) { err = "bath sites must be distinct and in range"; return PT_TEBD_EINVAL; }
    used[b.site] = 1;
    if (b.n_steps < 1 || !b.bond_dims || !b.tensors) { err = "bath needs n_steps >= 1, bond_dims and tensors"; return PT_TEBD_EINVAL; }
    if (b.bond_dims[0] != 1 && !b.initial) {
      err = "PT-MPO bond_dims[0] > 1 needs the site's initial augmented tensor";
      return PT_TEBD_EINVAL;
    }
    for (int k = 0; k <= b.n_steps; ++k)
      if (b.bond_dims[k] < 1 || b.bond_dims[k] > cfg->xi_max) { err = "PT-MPO bond dimension outside [1, xi_max]"; return PT_TEBD_EINVAL; }
    if (b.initial)
      for (int q = 0; q < 2 * 4 * b.bond_dims[0]; ++q)
        if (!std::isfinite(b.initial[q])) { err = "non-finite initial augmented tensor"; return PT_TEBD_EINVAL; }
    const int per = b.diagonal ? 4 : 16;
    for (int k = 0; k < b.n_steps; ++k) {
      if (!b.tensors[k]) { err = "null PT-MPO tensor"; return PT_TEBD_EINVAL; }
      const long long len = 2LL * b.bond_dims[k] * b.bond_dims[k + 1] * per;
      for (long long q = 0; q < len; ++q)
        if (!std::isfinite(b.tensors[k][q])) { err = "non-finite PT-MPO tensor entry"; return PT_TEBD_ENUMERIC; }
    }
  }
  return PT_TEBD_OK;
}

std::vector<long long> tensor_lengths(const pt_tebd_config* cfg) {
  std::vector<long long> out;
  for (int i = 0; i < cfg->n_baths; ++i) {
    const pt_tebd_bath& b = cfg->baths[i];
    long long t = 0;
    const int per = b.diagonal ? 4 : 16;
    for (int k = 0; k < b.n_steps; ++k) t += (long long)b.bond_dims[k] * b.bond_dims[k + 1] * per;
    out.push_back(std::max(t, 1LL));
  }
  return out;
}

std::vector<long long> cap_lengths(const pt_tebd_config* cfg) {
  std::vector<long long> out;
  for (int i = 0; i < cfg->n_baths; ++i) {
    const pt_tebd_bath& b = cfg->baths[i];
    long long t = 0;
    for (int k = 0; k <= b.n_steps; ++k) t += b.bond_dims[k];
    out.push_back(std::max(t, 1LL));
  }
  return out;
}

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

// ----------------------------------------------------------------- launch
// ------------------------------------------------ per-launch kernel timing
// When a handle has a timing class set, every launch of that class made
// while the handle is being advanced is bracketed by a pair of events on the
// handle's stream, and the kernels add their algorithmic flop counts to a
// device accumulator.
enum TimingClass : int { KT_NONE = 0, KT_EIGENSOLVER = 1, KT_BOND_GEMM = 2 };
thread_local pt_tebd* t_timing = nullptr;

// GEMM engines: VALU double (the original tile), matrix-core double, and
// matrix-core single precision for the mixed path's contractions
enum GemmEngine : int { GE_VALU = 0, GE_MFMA64 = 1, GE_MFMA32 = 2 };
thread_local int t_gemm_mixed = 0;   // set while a mixed-precision handle is stepped
thread_local int t_gemm_valu = 0;    // measurement switch: the VALU tile for every product
thread_local unsigned t_gemm_mixed_mask = ~(1u << 30);  // measurement switch: which single-precision kinds run single

// While a handle is advanced: its timing class and its GEMM engines.
struct TimingScope {
  pt_tebd* prev;
  int prev_mixed, prev_valu;
  unsigned prev_mask = ~(1u << 30);
  explicit TimingScope(pt_tebd* h)
      : prev(t_timing), prev_mixed(t_gemm_mixed), prev_valu(t_gemm_valu), prev_mask(t_gemm_mixed_mask) {
    t_timing = (h && h->timing_class) ? h : nullptr;
    t_gemm_mixed = (h && h->precision == PT_TEBD_FP32_MIXED) ? 1 : 0;
    t_gemm_valu = (h && h->gemm_valu) ? 1 : 0;
    t_gemm_mixed_mask = h ? h->mixed_mask : ~(1u << 30);
  }
  ~TimingScope() {
    t_timing = prev;
    t_gemm_mixed = prev_mixed;
    t_gemm_valu = prev_valu;
    t_gemm_mixed_mask = prev_mask;
  }
};

double* timed_flops(int cls) { return (t_timing && t_timing->timing_class == cls) ? t_timing->timing_flops : nullptr; }

bool timed_begin(int cls, hipStream_t st) {
  pt_tebd* h = t_timing;
  if (!h || h->timing_class != cls) return false;
  while (h->events.size() < h->events_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    h->events.push_back(e);
  }
  hipEventRecord(h->events[h->events_used], st);
  return true;
}

void timed_end(bool began, hipStream_t st) {
  if (!began) return;
  pt_tebd* h = t_timing;
  hipEventRecord(h->events[h->events_used + 1], st);
  h->events_used += 2;
}

void launch_gemm(hipStream_t st, const BondJob* jobs, int n_items, int kind, int subs, int m_cap, int n_cap) {
  dim3 grid((m_cap + ptt::GEMM_BM - 1) / ptt::GEMM_BM, (n_cap + ptt::GEMM_BN - 1) / ptt::GEMM_BN, n_items * subs);
  const bool single = t_gemm_mixed && ptt::gemm_kind_single(kind) && (t_gemm_mixed_mask >> kind & 1);
  const int engine = t_gemm_valu ? GE_VALU : single ? GE_MFMA32 : GE_MFMA64;
  const bool t = timed_begin(KT_BOND_GEMM, st);
  double* fl = timed_flops(KT_BOND_GEMM);
  if (engine == GE_VALU) ptt::k_bond_gemm<<<grid, ptt::GEMM_THREADS, 0, st>>>(jobs, kind, subs, fl);
  else if (engine == GE_MFMA64) ptt::k_bond_gemm_mfma<double><<<grid, ptt::GEMM_THREADS, 0, st>>>(jobs, kind, subs, fl);
  else ptt::k_bond_gemm_mfma<float><<<grid, ptt::GEMM_THREADS, 0, st>>>(jobs, kind, subs, fl);
  timed_end(t, st);
}

int elem_blocks(long long n);

// passes: block Gram-Schmidt passes of stage 6 (2), or 0 where the caller
// re-orthonormalises the vectors anyway (then only the column scaling)
void launch_heev(hipStream_t st, const HeevJob* jobs, int n_jobs, int n_cap, int passes = 2) {
  // the timed eigensolver region: tridiagonal reduction and stages 2-4
  const bool t = timed_begin(KT_EIGENSOLVER, st);
  ptt::heev_tridiag_kernel<<<n_jobs, ptt::HEEV_TRI_THREADS, 0, st>>>(jobs, timed_flops(KT_EIGENSOLVER));
  ptt::heev_solve_kernel<<<n_jobs, ptt::HEEV_SOLVE_THREADS, 0, st>>>(jobs);
  timed_end(t, st);
  dim3 grid((n_cap + ptt::HEEV_BT_COLS - 1) / ptt::HEEV_BT_COLS, n_jobs);
  const size_t shm = (size_t)n_cap * ptt::HEEV_BT_COLS * sizeof(double2);
  ptt::heev_backtransform_kernel<<<grid, ptt::HEEV_THREADS, shm, st>>>(jobs);
  const int tiles = (n_cap + ptt::GEMM_BM - 1) / ptt::GEMM_BM;
  const dim3 gg(tiles, tiles, n_jobs);
  const dim3 gn((n_cap + 63) / 64, n_jobs);
  if (passes == 0) {
    ptt::heev_orth_norm<<<gn, 256, 0, st>>>(jobs, 0, 1);
    return;
  }
  for (int pass = 0; pass < passes; ++pass) {
    ptt::heev_orth_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs, 0);
    ptt::heev_orth_mfix<<<dim3(elem_blocks((long long)n_cap * n_cap), n_jobs), kThreads, 0, st>>>(jobs);
    ptt::heev_orth_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs, 1);
    ptt::heev_orth_norm<<<gn, 256, 0, st>>>(jobs, 1, pass == passes - 1);
  }
}

int elem_blocks(long long n);

Exec exec_of(const pt_tebd* h) {
  return Exec{h->stream, h->cap, h->power_iters, h->cholqr, h->deflate, h->refine_levels, h->refine_tau};
}

// levels of block refinement of Gram-based singular values (refine.h)
void run_refine(const Exec& x, const ptt::RefineJob* R, const HeevJob* H, int n_jobs, int m_cap, int n_cap,
                int nh) {
  hipStream_t st = x.stream;
  const dim3 gnorm((nh + kThreads / 64 - 1) / (kThreads / 64), n_jobs);
  ptt::k_ref_norms<<<gnorm, kThreads, 0, st>>>(R);
  for (int level = 0; level < x.refine_levels; ++level) {
    ptt::k_ref_select<<<(n_jobs + 63) / 64, 64, 0, st>>>(R, n_jobs, x.refine_tau, level);
    dim3 gg((nh + ptt::GEMM_BM - 1) / ptt::GEMM_BM, (nh + ptt::GEMM_BN - 1) / ptt::GEMM_BN, n_jobs);
    ptt::k_ref_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(R, ptt::RK_GRAM);
    launch_heev(st, H, n_jobs, nh);
    dim3 gp((m_cap + ptt::GEMM_BM - 1) / ptt::GEMM_BM, (n_cap + ptt::GEMM_BN - 1) / ptt::GEMM_BN, n_jobs);
    ptt::k_ref_gemm<<<gp, ptt::GEMM_THREADS, 0, st>>>(R, ptt::RK_ROTP);
    dim3 gv((nh + ptt::GEMM_BM - 1) / ptt::GEMM_BM, (nh + ptt::GEMM_BN - 1) / ptt::GEMM_BN, n_jobs);
    ptt::k_ref_gemm<<<gv, ptt::GEMM_THREADS, 0, st>>>(R, ptt::RK_ROTV);
    ptt::k_ref_copy<<<dim3(elem_blocks((long long)m_cap * n_cap), n_jobs), kThreads, 0, st>>>(R);
    ptt::k_ref_norms<<<gnorm, kThreads, 0, st>>>(R);
  }
}

int elem_blocks(long long n) { return (int)std::min<long long>(std::max<long long>((n + kThreads - 1) / kThreads, 1), 1024); }

void run_sublayer(const Exec& x, const Sublayer& S, const ChainDev* chains) {
  const int n = (int)S.bonds.size();
  if (n == 0) return;
  const Caps& c = x.cap;
  hipStream_t st = x.stream;
  const long long rl = (long long)c.chi_cap * c.xi_cap;
  const int wide = (int)std::max<long long>(rl, c.nb);
  const BondJob* J = S.jobs;
  // (c)-(e): B_L, B_R, their Gram matrices, eigenpairs, singular values, ranks
  ptt::k_pack<<<dim3(elem_blocks(2 * rl * c.nb), n), kThreads, 0, st>>>(chains, J);
  launch_gemm(st, J, n, ptt::GK_GRAM_B, 2, c.nb, c.nb);
  launch_heev(st, S.heev_b, 2 * n, c.nh);
  launch_gemm(st, J, n, ptt::GK_PROD_B, 2, wide, wide);
  run_refine(x, S.ref_b, S.heev_ref_b, 2 * n, wide, wide, c.nb);
  ptt::k_rule_b<<<(n + 63) / 64, 64, 0, st>>>(J, n);
  ptt::k_form_xy<<<dim3(elem_blocks(2LL * c.nb * c.nb), n), kThreads, 0, st>>>(chains, J);
  // (e)-(f): D
  launch_gemm(st, J, n, ptt::GK_P, 1, c.dn, c.dn);
  // the gate stays in double precision on both paths (measurement switch:
  // bit 30 of PT_TEBD_MIXED_KINDS applies it in single precision)
  if (t_gemm_mixed && (t_gemm_mixed_mask >> 30 & 1)) ptt::k_apply_gate<float><<<dim3(elem_blocks((long long)c.nb * c.nb), n), kThreads, 0, st>>>(J);
  else ptt::k_apply_gate<double><<<dim3(elem_blocks((long long)c.nb * c.nb), n), kThreads, 0, st>>>(J);
  // (f)-(g): leading singular subspace of D
  ptt::k_sketch_init<<<dim3(elem_blocks((long long)c.dn * c.kc), n), kThreads, 0, st>>>(J);
  launch_gemm(st, J, n, ptt::GK_SKETCH, 1, c.dn, c.kc);
  auto copy_dim = [&](int dst, int src) { ptt::k_copy_dim<<<(n + 63) / 64, 64, 0, st>>>(J, n, dst, src, 1); };
  // second pass of an orthonormalisation: Cholesky QR, or the eigenvalue
  // form for the jobs it declines (dims[D_FB] = 0 for the others)
  auto second_pass = [&](const HeevJob* eig, const HeevJob* fallback) {
    if (x.cholqr) {
      ptt::k_chol_inv<<<n, ptt::CHOL_THREADS, 0, st>>>(J, ptt::D_GS, ptt::D_FB);
      launch_heev(st, fallback, n, c.kc);
    } else {
      launch_heev(st, eig, n, c.kc);
    }
  };
  auto defl_dims = [&](int stage, int side) {
    ptt::k_defl_dims<<<(n + 63) / 64, 64, 0, st>>>(J, n, stage, side);
  };
  auto df = [&](int op, int side, int m_cap, int n_cap) { launch_gemm(st, J, n, ptt::GK_DF + 2 * op + side, 1, m_cap, n_cap); };
  // Orthonormal basis of the sketch X (side 0: ya, rows M; side 1: za, rows
  // N).  Level 1: eigenvalues of X^H X with the numerical-rank rule
  // (directions below 1e-15 of the largest eigenvalue dropped), then a
  // Cholesky pass.  A Gram matrix resolves singular values only down to
  // ~3e-8 of the largest, so the dropped part is not noise in general:
  // level 2 takes the residual X - Q1 Q1^H X (two passes), orthonormalises it
  // the same way relative to its own scale (keeping singular values above
  // 1e-13 of the sketch's largest), against Q1 once more, and appends it.
  auto orth = [&](int side) {
    const int kb = side ? ptt::D_KZ : ptt::D_KQ;
    const HeevJob* h1 = side ? S.heev_oz : S.heev_oy;
    const HeevJob* h1b = side ? S.heev_ozb : S.heev_oyb;
    if (x.deflate) defl_dims(0, side);
    launch_gemm(st, J, n, side ? ptt::GK_GRAM_ZA : ptt::GK_GRAM_YA, 1, c.kc, c.kc);
    launch_heev(st, h1, n, c.kc, x.cholqr ? 0 : 2);
    if (x.deflate) defl_dims(1, side);
    launch_gemm(st, J, n, side ? ptt::GK_APPLY_ZA : ptt::GK_APPLY_YA, 1, c.dn, c.kc);
    copy_dim(ptt::D_GS, kb);
    launch_gemm(st, J, n, side ? ptt::GK_GRAM_ZB : ptt::GK_GRAM_YB, 1, c.kc, c.kc);
    second_pass(h1, h1b);
    if (!x.deflate) {
      launch_gemm(st, J, n, side ? ptt::GK_APPLY_ZB : ptt::GK_APPLY_YB, 1, c.dn, c.kc);
      return;
    }
    df(ptt::DF_APPLY1, side, c.dn, c.kc);  // Q1 into the scratch basis
    defl_dims(2, side);
    for (int pass = 0; pass < 2; ++pass) {
      df(ptt::DF_C, side, c.kc, c.kc);
      df(ptt::DF_R, side, c.dn, c.kc);
    }
    df(ptt::DF_GRAM2, side, c.kc, c.kc);
    launch_heev(st, S.heev_l2, n, c.kc);
    df(ptt::DF_APPLY2, side, c.dn, c.kc);
    df(ptt::DF_C2, side, c.kc, c.kc);
    df(ptt::DF_R2, side, c.dn, c.kc);
    defl_dims(3, side);
    df(ptt::DF_GRAM2B, side, c.kc, c.kc);
    if (x.cholqr) ptt::k_chol_inv<<<n, ptt::CHOL_THREADS, 0, st>>>(J, ptt::D_G2S, ptt::D_FB2);
    else copy_dim(ptt::D_FB2, ptt::D_G2S);
    launch_heev(st, S.heev_l2b, n, c.kc);
    df(ptt::DF_APPLY2B, side, c.dn, c.kc);
    defl_dims(4, side);
    ptt::k_defl_copy<<<dim3(elem_blocks((long long)c.dn * c.kc), n), kThreads, 0, st>>>(J, side);
  };
  orth(0);
  for (int it = 0; it < x.power_iters; ++it) {
    launch_gemm(st, J, n, ptt::GK_DH_Q, 1, c.dn, c.kc);
    copy_dim(ptt::D_GS, ptt::D_KQ);
    orth(1);
    launch_gemm(st, J, n, ptt::GK_D_Z, 1, c.dn, c.kc);
    copy_dim(ptt::D_GS, ptt::D_KZ);
    orth(0);
  }
  launch_gemm(st, J, n, ptt::GK_QH_D, 1, c.kc, c.dn);
  ptt::k_resid_copy<<<dim3(elem_blocks((long long)c.dn * c.dn), n), kThreads, 0, st>>>(J);
  launch_gemm(st, J, n, ptt::GK_RESID, 1, c.dn, c.dn);
  ptt::k_resid_partial<<<dim3(ptt::RESID_BLOCKS, n), kThreads, 0, st>>>(J);
  ptt::k_resid_norm<<<(n + 63) / 64, 64, 0, st>>>(J, n);
  ptt::k_copy_dim<<<(n + 63) / 64, 64, 0, st>>>(J, n, ptt::D_GS, ptt::D_KQ, 0);
  launch_gemm(st, J, n, ptt::GK_GRAM_BM, 1, c.kc, c.kc);
  launch_heev(st, S.heev_rr, n, c.kc);
  launch_gemm(st, J, n, ptt::GK_C, 1, c.kc, c.dn);
  run_refine(x, S.ref_d, S.heev_ref_d, n, c.kc, c.dn, c.kc);
  ptt::k_rule_d<<<(n + 63) / 64, 64, 0, st>>>(J, n);
  launch_gemm(st, J, n, ptt::GK_UD, 1, c.dn, c.chi_cap);
  ptt::k_scale_factors<<<dim3(elem_blocks(2LL * c.dn * c.chi_cap), n), kThreads, 0, st>>>(J);
  // (g)-(h): new site tensors
  launch_gemm(st, J, n, ptt::GK_NEWL, 1, (int)rl, 4 * c.chi_cap);
  ptt::k_store_gamma<<<dim3(elem_blocks(rl * 4 * c.chi_cap), n), kThreads, 0, st>>>(chains, J, 0);
  launch_gemm(st, J, n, ptt::GK_NEWR, 1, 4 * c.chi_cap, (int)rl);
  ptt::k_store_gamma<<<dim3(elem_blocks(rl * 4 * c.chi_cap), n), kThreads, 0, st>>>(chains, J, 1);
  ptt::k_finalize<<<n, kThreads, 0, st>>>(chains, J);
  ptt::k_logscale<<<1, 64, 0, st>>>(chains, J, n);
}

void run_half_step(pt_tebd* h, const ChainDev* chains) {
  const Exec x = exec_of(h);
  if (h->n_sites == 1) {
    ptt::k_apply_site_op<<<elem_blocks((long long)x.cap.chi_cap * x.cap.xi_cap * x.cap.chi_cap), kThreads, 0,
                           x.stream>>>(chains, 0, h->gates);
    return;
  }
  // E(dt/4) O(dt/2) E(dt/4) with 1-based bond parity: E = 0-based odd bonds
  run_sublayer(x, h->sub_even, chains);
  run_sublayer(x, h->sub_odd, chains);
  run_sublayer(x, h->sub_even, chains);
}

pt_tebd_status device_status(pt_tebd* h, int which) {
  int st = 0;
  if (!check(hipMemcpyAsync(&st, h->chain_host[which].status, sizeof(int), hipMemcpyDeviceToHost, h->stream), h,
             "status copy") ||
      !check(hipStreamSynchronize(h->stream), h, "stream sync"))
    return PT_TEBD_EDEVICE;
  if (st & ptt::ST_RANGE) { h->err = "PT-MPO step, bond dimension or work size out of range on the device"; return PT_TEBD_ERANGE; }
  if (st & (ptt::ST_NONFINITE | ptt::ST_ZERO)) { h->err = "non-finite value or zero norm during a bond update"; return PT_TEBD_ENUMERIC; }
  if (st & ptt::ST_EIG) { h->err = "eigensolver produced a non-finite value"; return PT_TEBD_ENUMERIC; }
  if (st & ptt::ST_NOCONV) { h->err = "eigensolver: the shifted factorisation of a nonzero Gram matrix never became definite"; return PT_TEBD_ENOCONV; }
  return PT_TEBD_OK;
}

void step_chain(pt_tebd* h, int which, int k) {
  const ChainDev* chains = h->chains + which;
  // the sublayer jobs index chain 0 of the array they are given
  run_half_step(h, chains);
  if (h->n_baths > 0) {
    ptt::k_pt_absorb<<<dim3(elem_blocks((long long)h->cap.chi_cap * 4 * h->cap.xi_cap * h->cap.chi_cap), h->n_baths),
                       kThreads, 0, h->stream>>>(chains, h->baths, k);
    ptt::k_pt_commit<<<1, 64 * ((h->n_baths + 63) / 64), 0, h->stream>>>(chains, h->baths, h->n_baths, k);
  }
  run_half_step(h, chains);
}

// observe on chain `which` at PT step `k`: fills host num/den/log
pt_tebd_status observe_raw(pt_tebd* h, int which, int k, int n_ops, const int* sites, const double* ovec_host,
                           std::vector<std::complex<double>>& num, std::vector<std::complex<double>>& den,
                           std::vector<double>& lg) {
  const ChainDev* chains = h->chains + which;
  const Caps& c = h->cap;
  ptt::k_obs_hat<<<dim3(elem_blocks((long long)c.chi_cap * 4 * c.chi_cap), c.n_sites), kThreads, 0, h->stream>>>(
      chains, h->baths, h->bath_of_site, k, h->obs);
  ptt::k_obs_scan<<<1, kThreads, 0, h->stream>>>(chains, h->obs);
  num.assign(n_ops, 0.0);
  den.assign(n_ops, 0.0);
  lg.assign(n_ops, 0.0);
  for (int off = 0; off < n_ops; off += h->ops_cap) {
    const int cnt = std::min(h->ops_cap, n_ops - off);
    if (!check(hipMemcpyAsync(h->ops_sites, sites + off, cnt * sizeof(int), hipMemcpyHostToDevice, h->stream), h, "ops copy") ||
        !check(hipMemcpyAsync(h->ops_vec, ovec_host + 8 * off, cnt * 4 * sizeof(double2), hipMemcpyHostToDevice, h->stream), h, "ops copy"))
      return PT_TEBD_EDEVICE;
    ptt::k_obs_ops<<<cnt, kThreads, 0, h->stream>>>(chains, h->obs, h->ops_sites, h->ops_vec, h->ops_out, h->ops_log);
    std::vector<double2> out(2 * cnt);
    std::vector<double> lgo(cnt);
    if (!check(hipMemcpyAsync(out.data(), h->ops_out, 2 * cnt * sizeof(double2), hipMemcpyDeviceToHost, h->stream), h, "ops out") ||
        !check(hipMemcpyAsync(lgo.data(), h->ops_log, cnt * sizeof(double), hipMemcpyDeviceToHost, h->stream), h, "ops out") ||
        !check(hipStreamSynchronize(h->stream), h, "stream sync"))
      return PT_TEBD_EDEVICE;
    for (int i = 0; i < cnt; ++i) {
      num[off + i] = {out[2 * i].x, out[2 * i].y};
      den[off + i] = {out[2 * i + 1].x, out[2 * i + 1].y};
      lg[off + i] = lgo[i];
    }
  }
  return device_status(h, which);
}

// observable vector o with o . vec(rho) = Tr[op rho]: o[i*d+j] = op[j][i]
void obs_vector(const double* op, double* o) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      o[2 * (i * 2 + j)] = op[2 * (j * 2 + i)];
      o[2 * (i * 2 + j) + 1] = op[2 * (j * 2 + i) + 1];
    }
}

void fill_heev(HeevJob& H, double2* a, int lda, int* n_ptr, double* w, double2* refl, double* tri, double* work,
               double* z, int n_cap, int* nvec, int rule, double eps, int capv, const double* extra, double rank_tol,
               double2* v, int ldv, int scale, int* status) {
  H.a = a; H.lda = lda; H.n_ptr = n_ptr; H.w = w; H.refl = refl; H.tri = tri; H.work = work; H.z = z;
  H.n_cap = n_cap; H.nvec_out = nvec; H.rule = rule; H.eps = eps; H.cap = capv; H.extra_tail = extra;
  H.rank_tol = rank_tol; H.v = v; H.ldv = ldv; H.scale = scale; H.status = status;
  H.noise_cluster = env_int("PT_TEBD_HEEV_NOISE", 1) != 0;
  H.abs_ref = nullptr;
  H.abs_tol = 0.0;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

pt_tebd_status pt_tebd_workspace_size(const pt_tebd_config* cfg, size_t* bytes) {
  std::string err;
  if (!bytes) return PT_TEBD_EINVAL;
  const pt_tebd_status s = validate(cfg, err);
  if (s != PT_TEBD_OK) return s;
  const Caps c = compute_caps(cfg, env_int("PT_TEBD_OVERSAMPLE", 64));
  *bytes = layout(c, cfg, tensor_lengths(cfg), cap_lengths(cfg), nullptr, nullptr);
  return PT_TEBD_OK;
}

namespace {
// message of the last failed pt_tebd_create on this thread
thread_local std::string t_create_error;

pt_tebd_status create_impl(const pt_tebd_config* cfg, void* ws, size_t bytes, void* stream, pt_tebd_t* out,
                           std::string& err) {
  if (!out) { err = "null output pointer"; return PT_TEBD_EINVAL; }
  *out = nullptr;
  pt_tebd_status s = validate(cfg, err);
  if (s != PT_TEBD_OK) return s;
  if (!ws) { err = "null workspace"; return PT_TEBD_EINVAL; }
  auto h = std::make_unique<pt_tebd>();
  struct KeepMessage {  // on failure the handle is freed: keep its message
    std::unique_ptr<pt_tebd>& h;
    std::string& err;
    ~KeepMessage() { if (h && !h->err.empty()) err = h->err; }
  } keep{h, err};
  h->oversample = std::max(8, env_int("PT_TEBD_OVERSAMPLE", 64));
  // two power iterations: with one, the leading subspace of D on the N = 21
  // workload at its chi cap is off by ~1e-6 in the observables.  The
  // FP32-mixed form is held to 1e-4, which one power iteration meets (the
  // block refinement of small singular values it still needs)
  const bool mixed = cfg->precision == PT_TEBD_FP32_MIXED;
  h->power_iters = std::max(0, env_int("PT_TEBD_POWER_ITERS", mixed ? 1 : 2));
  h->cholqr = env_int("PT_TEBD_CHOLQR", 1) != 0;
  // the Gram matrix of a sketch resolves directions down to ~3e-8 of its
  // largest singular value; truncation thresholds below 1e-8 need the
  // deflated second level of the range finder's orthonormalisation
  h->deflate = env_int("PT_TEBD_DEFLATE", cfg->svd_rel_cutoff < 1e-8 ? 1 : 0) != 0;
  // Gram matrices resolve singular values down to ~1e-8 of the largest,
  // which is where a truncation threshold eps ~ 1e-7 cuts: one level of
  // block refinement resolves the block below 1e-4 of the largest relative
  // to its own scale (down to ~1e-12); smaller thresholds take three
  h->refine_levels = std::max(0, env_int("PT_TEBD_REFINE_LEVELS", cfg->svd_rel_cutoff < 1e-8 ? 3 : 1));
  h->gemm_valu = env_int("PT_TEBD_GEMM_VALU", 0) != 0;
  h->mixed_mask = (unsigned)env_int("PT_TEBD_MIXED_KINDS", (int)~(1u << 30));
  h->cap = compute_caps(cfg, h->oversample);
  const Caps& c = h->cap;
  const auto tl = tensor_lengths(cfg), cl = cap_lengths(cfg);
  const size_t need = layout(c, cfg, tl, cl, nullptr, nullptr);
  if (bytes < need) { err = "workspace smaller than pt_tebd_workspace_size"; return PT_TEBD_ENOMEM; }
  DevPtrs P;
  layout(c, cfg, tl, cl, ws, &P);
  h->n_sites = cfg->n_sites;
  h->d = cfg->d;
  h->dt = cfg->dt;
  h->chi_max = cfg->chi_max;
  h->xi_max = cfg->xi_max;
  h->eps = cfg->svd_rel_cutoff;
  h->precision = cfg->precision;
  h->seed = cfg->seed;
  h->stream = static_cast<hipStream_t>(stream);
  h->ws = ws;
  h->ws_bytes = bytes;
  const int N = cfg->n_sites;
  hipStream_t st = h->stream;
  pt_tebd* hp = h.get();

  // chain propagators (host, double precision)
  std::vector<cplx> hs(4 * N), hb(16 * std::max(N - 1, 0)), lind;
  for (int i = 0; i < 4 * N; ++i) hs[i] = {cfg->h_site[2 * i], cfg->h_site[2 * i + 1]};
  for (size_t i = 0; i < hb.size(); ++i) hb[i] = {cfg->h_bond[2 * i], cfg->h_bond[2 * i + 1]};
  if (cfg->n_lindblad > 0) {
    lind.resize((size_t)N * cfg->n_lindblad * 4);
    for (size_t i = 0; i < lind.size(); ++i) lind[i] = {cfg->lindblad[2 * i], cfg->lindblad[2 * i + 1]};
  }
  h->gates_host = ptt::chain_gates(N, 2, cfg->dt, hs.data(), hb.data(), cfg->n_lindblad, lind.data());
  std::vector<double2> gbuf;
  for (const auto& g : h->gates_host)
    for (const auto& z : g) gbuf.push_back(ptt::mk<double>(z.real(), z.imag()));
  if (!check(hipMemcpyAsync(P.gates, gbuf.data(), gbuf.size() * sizeof(double2), hipMemcpyHostToDevice, st), hp, "gates") ||
      !check(hipStreamSynchronize(st), hp, "gates sync"))
    return PT_TEBD_EDEVICE;
  h->gates = P.gates;

  // chain state: product initial state, Gamma_n[0][s][0][0] = vec(rho_n)[s]
  for (int k = 0; k < 2; ++k) {
    ChainDev& C = h->chain_host[k];
    C.n_sites = N; C.chi_cap = c.chi_cap; C.xi_cap = c.xi_cap; C.gam_cap = c.gam_cap;
    C.gam = P.gam[k]; C.parity = P.parity[k]; C.chi = P.chi[k]; C.xi = P.xi[k];
    C.lam = P.lam[k]; C.log_scale = P.log_scale[k]; C.status = P.status[k]; C.work = P.work[k];
  }
  {
    std::vector<double2> g0((size_t)N * 2 * c.gam_cap, ptt::mk<double>(0.0, 0.0));
    for (int n = 0; n < N; ++n)
      for (int s2 = 0; s2 < 4; ++s2)
        g0[(size_t)n * 2 * c.gam_cap + s2] = ptt::mk<double>(cfg->rho0[8 * n + 2 * s2], cfg->rho0[8 * n + 2 * s2 + 1]);
    std::vector<int> zeros(N, 0), ones(N + 1, 1), xi0(N, 1);
    // correlated starts: Gamma_n[0][s][e][0] = R[s][e] (compact [a][s][e][b])
    for (int i = 0; i < cfg->n_baths; ++i) {
      const pt_tebd_bath& b = cfg->baths[i];
      if (!b.initial) continue;
      const int x0 = b.bond_dims[0];
      xi0[b.site] = x0;
      for (int s2 = 0; s2 < 4; ++s2)
        for (int e = 0; e < x0; ++e)
          g0[(size_t)b.site * 2 * c.gam_cap + (size_t)s2 * x0 + e] =
              ptt::mk<double>(b.initial[2 * (s2 * x0 + e)], b.initial[2 * (s2 * x0 + e) + 1]);
    }
    std::vector<double> lam((size_t)(N + 1) * c.chi_cap, 0.0);
    for (int n = 0; n <= N; ++n) lam[(size_t)n * c.chi_cap] = 1.0;
    double zero = 0.0;
    const double zw[4] = {0.0, 0.0, 0.0, 0.0};
    int zi = 0;
    bool ok = check(hipMemcpyAsync(P.gam[0], g0.data(), g0.size() * sizeof(double2), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.parity[0], zeros.data(), N * sizeof(int), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.chi[0], ones.data(), (N + 1) * sizeof(int), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.xi[0], xi0.data(), N * sizeof(int), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.lam[0], lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.log_scale[0], &zero, sizeof(double), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.status[0], &zi, sizeof(int), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.status[1], &zi, sizeof(int), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.work[0], zw, sizeof(zw), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.work[1], zw, sizeof(zw), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipMemcpyAsync(P.chains, h->chain_host, 2 * sizeof(ChainDev), hipMemcpyHostToDevice, st), hp, "init") &&
              check(hipStreamSynchronize(st), hp, "init sync");
    if (!ok) return PT_TEBD_EDEVICE;
  }
  h->chains = P.chains;

  // baths: tensors, offsets, dims, caps (backward recursion when not given)
  h->n_baths = cfg->n_baths;
  h->bath_of_site_host.assign(N, -1);
  h->pt_steps = 1 << 30;
  std::vector<BathDev> bdev(std::max(cfg->n_baths, 1));
  for (int i = 0; i < cfg->n_baths; ++i) {
    const pt_tebd_bath& b = cfg->baths[i];
    const int m = b.n_steps, per = b.diagonal ? 4 : 16;
    h->pt_steps = std::min(h->pt_steps, m);
    h->bath_of_site_host[b.site] = i;
    std::vector<double2> tens;
    std::vector<long long> toff(m);
    std::vector<std::vector<cplx>> thost(m);
    std::vector<int> dims(b.bond_dims, b.bond_dims + m + 1);
    for (int k = 0; k < m; ++k) {
      toff[k] = (long long)tens.size();
      const long long len = (long long)dims[k] * dims[k + 1] * per;
      thost[k].resize(len);
      for (long long q = 0; q < len; ++q) {
        tens.push_back(ptt::mk<double>(b.tensors[k][2 * q], b.tensors[k][2 * q + 1]));
        thost[k][q] = {b.tensors[k][2 * q], b.tensors[k][2 * q + 1]};
      }
    }
    std::vector<double2> caps;
    std::vector<long long> coff(m + 1);
    std::vector<std::vector<cplx>> chost;
    if (!b.caps) chost = ptt::caps_backward(thost, dims, 2, b.diagonal != 0);
    for (int k = 0; k <= m; ++k) {
      coff[k] = (long long)caps.size();
      for (int e = 0; e < dims[k]; ++e) {
        if (b.caps) caps.push_back(ptt::mk<double>(b.caps[k][2 * e], b.caps[k][2 * e + 1]));
        else caps.push_back(ptt::mk<double>(chost[k][e].real(), chost[k][e].imag()));
      }
    }
    bool ok = check(hipMemcpyAsync(P.bath_tens[i], tens.data(), tens.size() * sizeof(double2), hipMemcpyHostToDevice, st), hp, "bath") &&
              check(hipMemcpyAsync(P.bath_toff[i], toff.data(), m * sizeof(long long), hipMemcpyHostToDevice, st), hp, "bath") &&
              check(hipMemcpyAsync(P.bath_dims[i], dims.data(), (m + 1) * sizeof(int), hipMemcpyHostToDevice, st), hp, "bath") &&
              check(hipMemcpyAsync(P.bath_caps[i], caps.data(), caps.size() * sizeof(double2), hipMemcpyHostToDevice, st), hp, "bath") &&
              check(hipMemcpyAsync(P.bath_coff[i], coff.data(), (m + 1) * sizeof(long long), hipMemcpyHostToDevice, st), hp, "bath") &&
              check(hipStreamSynchronize(st), hp, "bath sync");
    if (!ok) return PT_TEBD_EDEVICE;
    BathDev& bd = bdev[i];
    bd.site = b.site; bd.n_steps = m; bd.diagonal = b.diagonal ? 1 : 0;
    bd.tens = P.bath_tens[i]; bd.toff = P.bath_toff[i]; bd.dims = P.bath_dims[i];
    bd.caps = P.bath_caps[i]; bd.coff = P.bath_coff[i];
  }
  if (cfg->n_baths == 0) h->pt_steps = 1 << 30;
  if (!check(hipMemcpyAsync(P.baths, bdev.data(), bdev.size() * sizeof(BathDev), hipMemcpyHostToDevice, st), hp, "baths") ||
      !check(hipMemcpyAsync(P.bath_of_site, h->bath_of_site_host.data(), N * sizeof(int), hipMemcpyHostToDevice, st), hp, "baths") ||
      !check(hipStreamSynchronize(st), hp, "sync"))
    return PT_TEBD_EDEVICE;
  h->baths = P.baths;
  h->bath_of_site = P.bath_of_site;
  h->obs = P.obs;
  h->ops_cap = 8 * N + 8;
  h->ops_sites = P.ops_sites;
  h->ops_vec = P.ops_vec;
  h->ops_out = P.ops_out;
  h->ops_log = P.ops_log;
  h->site_op = P.site_op;
  h->timing_flops = P.timing_flops;

  // measurement switch PT_TEBD_MIXED_FLOOR: the mixed form's noise floor in units of u_32
  const char* mf = std::getenv("PT_TEBD_MIXED_FLOOR");
  const double mixed_floor_units = (mf && *mf) ? std::atof(mf) : 1.0;
  // sublayer job tables
  for (int par = 0; par < 2; ++par) {
    Sublayer& S = par == 0 ? h->sub_even : h->sub_odd;
    for (int b = (par == 0 ? 1 : 0); b + 1 < N; b += 2) S.bonds.push_back(b);
    const int n = (int)S.bonds.size();
    S.jobs = P.jobs[par];
    S.heev_b = P.hb[par];
    S.heev_oy = P.hoy[par];
    S.heev_oz = P.hoz[par];
    S.heev_oyb = P.hoyb[par];
    S.heev_ozb = P.hozb[par];
    S.heev_l2 = P.hl2[par];
    S.heev_l2b = P.hl2b[par];
    S.heev_rr = P.hrr[par];
    S.ref_b = P.rb[par];
    S.ref_d = P.rd[par];
    S.heev_ref_b = P.hrb[par];
    S.heev_ref_d = P.hrd[par];
    std::vector<HeevJob> hb2(2 * std::max(n, 1)), hoy(std::max(n, 1)), hoz(std::max(n, 1)), hrr(std::max(n, 1));
    std::vector<HeevJob> hoyb(std::max(n, 1)), hozb(std::max(n, 1)), hl2(std::max(n, 1)), hl2b(std::max(n, 1));
    std::vector<HeevJob> hrb(2 * std::max(n, 1)), hrd(std::max(n, 1));
    std::vector<ptt::RefineJob> rb(2 * std::max(n, 1)), rd(std::max(n, 1));
    for (int i = 0; i < n; ++i) {
      BondJob J = P.slots[i];
      J.chain = 0;
      J.bond = S.bonds[i];
      J.gate = P.gates + (size_t)J.bond * 256;
      J.chi_max = cfg->chi_max;
      J.k_cap = c.kc;
      J.k_sketch = c.ks;
      J.eps = cfg->svd_rel_cutoff;
      // single-precision contractions resolve singular values down to about
      // u_32 = 2^-24 of the matrix's Frobenius norm
      J.floor_rel = (cfg->precision == PT_TEBD_FP32_MIXED) ? mixed_floor_units * 5.9604644775390625e-8 : 0.0;
      J.seed = ptt::splitmix64(cfg->seed ^ (0xA24BAED4963EE407ull * (unsigned long long)(J.bond + 1)));
      J.nb_cap = c.nb;
      J.dn_cap = c.dn;
      J.ldr = std::max(c.chi_cap * c.xi_cap, c.nb);
      S.host_jobs.push_back(J);
      int* st0 = J.estat;  // folded into the stepped chain's status by k_finalize
      fill_heev(hb2[2 * i], J.gl, c.nb, J.dims + ptt::D_NL, J.wl, P.h_refl[0][i], P.h_tri[0][i], P.h_work[0][i],
                P.h_z[0][i], c.nh, J.dims + ptt::D_L, ptt::RULE_FULL, J.eps, 0, nullptr, 0.0, J.vl, c.nb,
                ptt::SCALE_NONE, st0);
      fill_heev(hb2[2 * i + 1], J.gr, c.nb, J.dims + ptt::D_NR, J.wr, P.h_refl[1][i], P.h_tri[1][i], P.h_work[1][i],
                P.h_z[1][i], c.nh, J.dims + ptt::D_R, ptt::RULE_FULL, J.eps, 0, nullptr, 0.0, J.vr, c.nb,
                ptt::SCALE_NONE, st0);
      fill_heev(hoy[i], J.gk, c.kc, J.dims + ptt::D_GS, J.wk, P.h_refl[0][i], P.h_tri[0][i], P.h_work[0][i],
                P.h_z[0][i], c.nh, J.dims + ptt::D_KQ, ptt::RULE_RANK, 0.0, 0, nullptr, 1e-15, J.vk, c.kc,
                ptt::SCALE_INV_SQRT, st0);
      hoz[i] = hoy[i];
      hoz[i].nvec_out = J.dims + ptt::D_KZ;
      hoyb[i] = hoy[i];
      hoyb[i].n_ptr = J.dims + ptt::D_FB;
      hozb[i] = hoz[i];
      hozb[i].n_ptr = J.dims + ptt::D_FB;
      // deflation level 2: residual directions above 1e-26 of the level-1
      // basis's largest Gram eigenvalue (singular values above 1e-13 of it)
      hl2[i] = hoy[i];
      hl2[i].n_ptr = J.dims + ptt::D_GS2;
      hl2[i].nvec_out = J.dims + ptt::D_K2;
      hl2[i].abs_ref = J.norms + 4;
      hl2[i].abs_tol = 1e-26;
      hl2b[i] = hoy[i];
      hl2b[i].n_ptr = J.dims + ptt::D_FB2;
      hl2b[i].nvec_out = J.dims + ptt::D_K2;
      fill_heev(hrr[i], J.gk, c.kc, J.dims + ptt::D_GS, J.wk, P.h_refl[0][i], P.h_tri[0][i], P.h_work[0][i],
                P.h_z[0][i], c.nh, J.dims + ptt::D_CHI, ptt::RULE_FULL, J.eps, cfg->chi_max, J.norms + 2, 0.0,
                J.vk, c.kc, ptt::SCALE_NONE, st0);
      int* blk = P.blk[i];
      // B_L: columns of pl (rl x n) on side 0, rows of pl (n x cl) on side 1
      ptt::RefineJob& RL = rb[2 * i];
      RL = ptt::RefineJob{};
      RL.P = J.pl; RL.ldp = c.nb; RL.ldp_ptr = nullptr; RL.cols = 0; RL.side_ptr = J.dims + ptt::D_SL; RL.side_cols = 0;
      RL.len_cols = J.dims + ptt::D_RL; RL.len_rows = J.dims + ptt::D_CL; RL.n_ptr = J.dims + ptt::D_NL;
      RL.V = J.vl; RL.ldv = c.nb; RL.nv_ptr = J.dims + ptt::D_NL; RL.s = J.sl; RL.blk = blk;
      RL.G = J.gl; RL.ldg = c.nb; RL.W = J.x; RL.ldw = c.nb; RL.TP = J.tpl; RL.ldtp = c.nb; RL.TV = J.tvl; RL.ldtv = c.nb;
      // B_R: rows of pr (n x cr) on side 0, columns of pr (rr x n) on side 1
      ptt::RefineJob& RR = rb[2 * i + 1];
      RR = ptt::RefineJob{};
      RR.P = J.pr; RR.ldp = J.ldr; RR.ldp_ptr = nullptr; RR.cols = 0; RR.side_ptr = J.dims + ptt::D_SR; RR.side_cols = 1;
      RR.len_cols = J.dims + ptt::D_RR; RR.len_rows = J.dims + ptt::D_CR; RR.n_ptr = J.dims + ptt::D_NR;
      RR.V = J.vr; RR.ldv = c.nb; RR.nv_ptr = J.dims + ptt::D_NR; RR.s = J.sr; RR.blk = blk + 2;
      RR.G = J.gr; RR.ldg = c.nb; RR.W = J.y; RR.ldw = c.nb; RR.TP = J.tpr; RR.ldtp = J.ldr; RR.TV = J.tvr; RR.ldtv = c.nb;
      // D: rows of vdh = W^H Q^H D (KQ x N, leading dim N)
      ptt::RefineJob& RD = rd[i];
      RD = ptt::RefineJob{};
      RD.P = J.vdh; RD.ldp = 0; RD.ldp_ptr = J.dims + ptt::D_N; RD.cols = 0; RD.side_ptr = nullptr;
      RD.len_cols = J.dims + ptt::D_N; RD.len_rows = J.dims + ptt::D_N; RD.n_ptr = J.dims + ptt::D_KQ;
      RD.V = J.vk; RD.ldv = c.kc; RD.nv_ptr = J.dims + ptt::D_KQ; RD.s = J.sk; RD.blk = blk + 4;
      RD.G = J.gk; RD.ldg = c.kc; RD.W = J.omega; RD.ldw = c.kc; RD.TP = J.za; RD.ldtp = c.dn; RD.TV = J.zb; RD.ldtv = c.kc;
      fill_heev(hrb[2 * i], J.gl, c.nb, blk + 1, J.wl, P.h_refl[0][i], P.h_tri[0][i], P.h_work[0][i], P.h_z[0][i],
                c.nh, J.dims + ptt::D_L, ptt::RULE_FULL, 0.0, 0, nullptr, 0.0, J.x, c.nb, ptt::SCALE_NONE, st0);
      fill_heev(hrb[2 * i + 1], J.gr, c.nb, blk + 3, J.wr, P.h_refl[1][i], P.h_tri[1][i], P.h_work[1][i],
                P.h_z[1][i], c.nh, J.dims + ptt::D_R, ptt::RULE_FULL, 0.0, 0, nullptr, 0.0, J.y, c.nb,
                ptt::SCALE_NONE, st0);
      fill_heev(hrd[i], J.gk, c.kc, blk + 5, J.wk, P.h_refl[0][i], P.h_tri[0][i], P.h_work[0][i], P.h_z[0][i],
                c.nh, J.dims + ptt::D_CHI, ptt::RULE_FULL, 0.0, 0, nullptr, 0.0, J.omega, c.kc, ptt::SCALE_NONE, st0);
    }
    if (n > 0) {
      bool ok = check(hipMemcpyAsync(S.jobs, S.host_jobs.data(), n * sizeof(BondJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_b, hb2.data(), 2 * n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_oy, hoy.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_oz, hoz.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_oyb, hoyb.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_ozb, hozb.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_l2, hl2.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_l2b, hl2b.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_rr, hrr.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_ref_b, hrb.data(), 2 * n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.heev_ref_d, hrd.data(), n * sizeof(HeevJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.ref_b, rb.data(), 2 * n * sizeof(ptt::RefineJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipMemcpyAsync(S.ref_d, rd.data(), n * sizeof(ptt::RefineJob), hipMemcpyHostToDevice, st), hp, "jobs") &&
                check(hipStreamSynchronize(st), hp, "jobs sync");
      if (!ok) return PT_TEBD_EDEVICE;
    }
  }
  *out = h.release();
  return PT_TEBD_OK;
}
}  // namespace

pt_tebd_status pt_tebd_create(const pt_tebd_config* cfg, void* ws, size_t bytes, void* stream, pt_tebd_t* out) {
  std::string err;
  const pt_tebd_status s = create_impl(cfg, ws, bytes, stream, out, err);
  t_create_error = (s == PT_TEBD_OK) ? std::string() : err;
  return s;
}

pt_tebd_status pt_tebd_step(pt_tebd_t h, int32_t n_steps) {
  if (!h || n_steps < 0) return PT_TEBD_EINVAL;
  if (h->n_baths > 0 && h->step + n_steps > h->pt_steps) {
    h->err = "stepping past the end of a PT-MPO";
    return PT_TEBD_ERANGE;
  }
  TimingScope timing(h);
  for (int i = 0; i < n_steps; ++i) {
    step_chain(h, 0, h->step + 1);
    ++h->step;
  }
  if (!check(hipGetLastError(), h, "kernel launch")) return PT_TEBD_EDEVICE;
  return PT_TEBD_OK;
}

pt_tebd_status pt_tebd_observe(pt_tebd_t h, int32_t n_ops, const int32_t* sites, const double* ops, double* out,
                               double* trace_out) {
  if (!h || n_ops < 0 || (n_ops > 0 && (!sites || !ops || !out))) return PT_TEBD_EINVAL;
  for (int i = 0; i < n_ops; ++i)
    if (sites[i] < 0 || sites[i] >= h->n_sites) { h->err = "observable site out of range"; return PT_TEBD_EINVAL; }
  for (int i = 0; i < 8 * n_ops; ++i)
    if (!std::isfinite(ops[i])) { h->err = "non-finite operator"; return PT_TEBD_EINVAL; }
  // one extra trace request at site 0 so the trace is always available
  std::vector<int> s2(sites, sites + n_ops);
  std::vector<double> ov(8 * (n_ops + 1));
  for (int i = 0; i < n_ops; ++i) obs_vector(ops + 8 * i, ov.data() + 8 * i);
  s2.push_back(0);
  const double eye[8] = {1, 0, 0, 0, 0, 0, 1, 0};
  obs_vector(eye, ov.data() + 8 * n_ops);
  std::vector<std::complex<double>> num, den;
  std::vector<double> lg;
  const pt_tebd_status s = observe_raw(h, 0, h->step, n_ops + 1, s2.data(), ov.data(), num, den, lg);
  if (s != PT_TEBD_OK) return s;
  for (int i = 0; i < n_ops; ++i) {
    const std::complex<double> v = num[i] / den[i];
    out[2 * i] = v.real();
    out[2 * i + 1] = v.imag();
  }
  if (trace_out) {
    const std::complex<double> t = std::exp(lg[n_ops]) * num[n_ops];
    trace_out[0] = t.real();
    trace_out[1] = t.imag();
  }
  return PT_TEBD_OK;
}

namespace {
// one insertion of a multi-time correlation: at step offset m the
// super-operator of op acts on site from the left (side 0: C rho) or from
// the right (side 1: rho C)
struct Insertion {
  int m, site, side;
  const double* op;
};

// site super-operator in the site-major vec convention (row index i*2+j of
// rho_ij): left  (C rho)_ij = sum_k C_ik rho_kj,  right (rho C)_ij = sum_l rho_il C_lj
void site_superop(const double* op, int side, std::vector<double2>& sop) {
  sop.assign(16, ptt::mk<double>(0.0, 0.0));
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) {
          double re = 0, im = 0;
          if (side == 0 && j == l) { re = op[2 * (i * 2 + k)]; im = op[2 * (i * 2 + k) + 1]; }
          if (side == 1 && i == k) { re = op[2 * (l * 2 + j)]; im = op[2 * (l * 2 + j) + 1]; }
          sop[(i * 2 + j) * 4 + (k * 2 + l)] = ptt::mk<double>(re, im);
        }
}

// Appendix A.4, eq. two-time-corr-decomposed generalised to P insertions:
// fork the augmented state at the current step, apply the insertions at
// their offsets (stepping the fork in between), then read Tr[B X] at offsets
// m_P + j, j = 0..n_steps, divided by Tr rho at the fork step.
pt_tebd_status correlate_impl(pt_tebd* h, const std::vector<Insertion>& ins, int32_t site_b, const double* op_b,
                              int32_t n_steps, double* out) {
  if (!op_b || !out || n_steps < 0 || ins.empty()) return PT_TEBD_EINVAL;
  if (site_b < 0 || site_b >= h->n_sites) return PT_TEBD_EINVAL;
  int last = 0;
  for (const Insertion& p : ins) {
    if (!p.op || p.site < 0 || p.site >= h->n_sites || p.m < last || (p.side != 0 && p.side != 1)) {
      h->err = "insertions need sites in range, sides 0 or 1 and non-decreasing offsets from 0";
      return PT_TEBD_EINVAL;
    }
    last = p.m;
    for (int i = 0; i < 8; ++i)
      if (!std::isfinite(p.op[i])) { h->err = "non-finite operator"; return PT_TEBD_EINVAL; }
  }
  for (int i = 0; i < 8; ++i)
    if (!std::isfinite(op_b[i])) { h->err = "non-finite operator"; return PT_TEBD_EINVAL; }
  if (h->n_baths > 0 && h->step + last + n_steps > h->pt_steps) {
    h->err = "correlation runs past the end of a PT-MPO";
    return PT_TEBD_ERANGE;
  }
  TimingScope timing(h);
  // trace of the main state at the fork step
  const double eye[8] = {1, 0, 0, 0, 0, 0, 1, 0};
  double ov[8];
  obs_vector(eye, ov);
  int s0 = 0;
  std::vector<std::complex<double>> num, den;
  std::vector<double> lg;
  pt_tebd_status s = observe_raw(h, 0, h->step, 1, &s0, ov, num, den, lg);
  if (s != PT_TEBD_OK) return s;
  const std::complex<double> tr0 = num[0];
  const double tr0_log = lg[0];
  // fork: copy the whole main state into the second chain slot
  const ChainDev& M = h->chain_host[0];
  const ChainDev& F = h->chain_host[1];
  const int N = h->n_sites;
  const Caps& c = h->cap;
  bool ok = check(hipMemcpyAsync(F.gam, M.gam, (size_t)N * 2 * c.gam_cap * sizeof(double2), hipMemcpyDeviceToDevice, h->stream), h, "fork") &&
            check(hipMemcpyAsync(F.parity, M.parity, N * sizeof(int), hipMemcpyDeviceToDevice, h->stream), h, "fork") &&
            check(hipMemcpyAsync(F.chi, M.chi, (N + 1) * sizeof(int), hipMemcpyDeviceToDevice, h->stream), h, "fork") &&
            check(hipMemcpyAsync(F.xi, M.xi, N * sizeof(int), hipMemcpyDeviceToDevice, h->stream), h, "fork") &&
            check(hipMemcpyAsync(F.lam, M.lam, (size_t)(N + 1) * c.chi_cap * sizeof(double), hipMemcpyDeviceToDevice, h->stream), h, "fork") &&
            check(hipMemcpyAsync(F.log_scale, M.log_scale, sizeof(double), hipMemcpyDeviceToDevice, h->stream), h, "fork") &&
            check(hipMemsetAsync(F.status, 0, sizeof(int), h->stream), h, "fork");
  if (!ok) return PT_TEBD_EDEVICE;
  int offset = 0;
  std::vector<double2> sop;
  for (const Insertion& p : ins) {
    for (int k = offset; k < p.m; ++k) step_chain(h, 1, h->step + k + 1);
    offset = p.m;
    site_superop(p.op, p.side, sop);
    if (!check(hipMemcpyAsync(h->site_op, sop.data(), 16 * sizeof(double2), hipMemcpyHostToDevice, h->stream), h, "op") ||
        !check(hipStreamSynchronize(h->stream), h, "op sync"))
      return PT_TEBD_EDEVICE;
    ptt::k_apply_site_op<<<elem_blocks((long long)c.chi_cap * c.xi_cap * c.chi_cap), kThreads, 0, h->stream>>>(
        h->chains + 1, p.site, h->site_op);
  }
  double obv[8];
  obs_vector(op_b, obv);
  for (int j = 0; j <= n_steps; ++j) {
    if (j > 0) step_chain(h, 1, h->step + offset + j);
    s = observe_raw(h, 1, h->step + offset + j, 1, &site_b, obv, num, den, lg);
    if (s != PT_TEBD_OK) return s;
    const std::complex<double> v = num[0] * std::exp(lg[0] - tr0_log) / tr0;
    out[2 * j] = v.real();
    out[2 * j + 1] = v.imag();
  }
  return PT_TEBD_OK;
}
}  // namespace

pt_tebd_status pt_tebd_correlate(pt_tebd_t h, int32_t site_a, const double* op_a, int32_t site_b,
                                 const double* op_b, int32_t n_steps, double* out) {
  if (!h || !op_a) return PT_TEBD_EINVAL;
  return correlate_impl(h, {Insertion{0, site_a, 0, op_a}}, site_b, op_b, n_steps, out);
}

pt_tebd_status pt_tebd_fdt_spectra(pt_tebd_t h, int32_t site, const double* op, int32_t n_steps, int32_t n_omega,
                                   const double* omega, double* corr, double* s_out, double* chi_out) {
  if (!h || !op || !omega || !corr || !s_out || !chi_out || n_omega < 1 || n_steps < 0) return PT_TEBD_EINVAL;
  for (int i = 0; i < 4; ++i)  // Hermitian: op = op^H
    if (std::fabs(op[2 * i] - op[2 * ((i % 2) * 2 + i / 2)]) > 1e-12 * (1.0 + std::fabs(op[2 * i])) ||
        std::fabs(op[2 * i + 1] + op[2 * ((i % 2) * 2 + i / 2) + 1]) > 1e-12 * (1.0 + std::fabs(op[2 * i + 1]))) {
      h->err = "the spectra need a Hermitian operator";
      return PT_TEBD_EINVAL;
    }
  pt_tebd_status s = correlate_impl(h, {Insertion{0, site, 0, op}}, site, op, n_steps, corr);
  if (s != PT_TEBD_OK) return s;
  double2* dc = nullptr;
  double *dw = nullptr, *ds = nullptr, *dx = nullptr;
  bool ok = check(hipMalloc(&dc, (n_steps + 1) * sizeof(double2)), h, "spectra") &&
            check(hipMalloc(&dw, n_omega * sizeof(double)), h, "spectra") &&
            check(hipMalloc(&ds, n_omega * sizeof(double)), h, "spectra") &&
            check(hipMalloc(&dx, n_omega * sizeof(double)), h, "spectra") &&
            check(hipMemcpyAsync(dc, corr, (n_steps + 1) * sizeof(double2), hipMemcpyHostToDevice, h->stream), h, "spectra") &&
            check(hipMemcpyAsync(dw, omega, n_omega * sizeof(double), hipMemcpyHostToDevice, h->stream), h, "spectra");
  if (ok) {
    ptt::k_fdt_spectra<<<(n_omega + 255) / 256, 256, 0, h->stream>>>(dc, n_steps, h->dt, dw, n_omega, ds, dx);
    ok = check(hipGetLastError(), h, "spectra") &&
         check(hipMemcpyAsync(s_out, ds, n_omega * sizeof(double), hipMemcpyDeviceToHost, h->stream), h, "spectra") &&
         check(hipMemcpyAsync(chi_out, dx, n_omega * sizeof(double), hipMemcpyDeviceToHost, h->stream), h, "spectra") &&
         check(hipStreamSynchronize(h->stream), h, "spectra");
  }
  (void)hipFree(dc); (void)hipFree(dw); (void)hipFree(ds); (void)hipFree(dx);
  return ok ? PT_TEBD_OK : PT_TEBD_EDEVICE;
}

pt_tebd_status pt_tebd_correlate_multi(pt_tebd_t h, int32_t n_ins, const int32_t* offsets, const int32_t* sites,
                                       const double* ops, const int32_t* sides, int32_t site_b, const double* op_b,
                                       int32_t n_steps, double* out) {
  if (!h || n_ins < 1 || !offsets || !sites || !ops || !sides) return PT_TEBD_EINVAL;
  std::vector<Insertion> ins(n_ins);
  for (int p = 0; p < n_ins; ++p) ins[p] = Insertion{offsets[p], sites[p], sides[p], ops + 8 * p};
  return correlate_impl(h, ins, site_b, op_b, n_steps, out);
}

pt_tebd_status pt_tebd_bond_dims(pt_tebd_t h, int32_t* chi, int32_t* xi) {
  if (!h || !chi) return PT_TEBD_EINVAL;
  const int N = h->n_sites;
  std::vector<int> c(N + 1), x(N);
  if (!check(hipMemcpyAsync(c.data(), h->chain_host[0].chi, (N + 1) * sizeof(int), hipMemcpyDeviceToHost, h->stream), h, "dims") ||
      !check(hipMemcpyAsync(x.data(), h->chain_host[0].xi, N * sizeof(int), hipMemcpyDeviceToHost, h->stream), h, "dims") ||
      !check(hipStreamSynchronize(h->stream), h, "sync"))
    return PT_TEBD_EDEVICE;
  for (int b = 0; b + 1 < N; ++b) chi[b] = c[b + 1];
  if (xi)
    for (int n = 0; n < N; ++n) xi[n] = x[n];
  return device_status(h, 0);
}

pt_tebd_status pt_tebd_model_flops(pt_tebd_t h, double* out, int32_t reset) {
  if (!h || !out) return PT_TEBD_EINVAL;
  double w[4];
  if (!check(hipMemcpyAsync(w, h->chain_host[0].work, sizeof(w), hipMemcpyDeviceToHost, h->stream), h, "work") ||
      !check(hipStreamSynchronize(h->stream), h, "sync"))
    return PT_TEBD_EDEVICE;
  for (int i = 0; i < 4; ++i) out[i] = w[i];
  if (reset) {
    const double z[4] = {0.0, 0.0, 0.0, 0.0};
    if (!check(hipMemcpyAsync(h->chain_host[0].work, z, sizeof(z), hipMemcpyHostToDevice, h->stream), h, "work") ||
        !check(hipStreamSynchronize(h->stream), h, "sync"))
      return PT_TEBD_EDEVICE;
  }
  return PT_TEBD_OK;
}

namespace {
// bytes of a snapshot: header, Gamma buffers, parity, chi, xi, lambda, log-scale
size_t snapshot_bytes(const pt_tebd* h) {
  const int N = h->n_sites;
  const Caps& c = h->cap;
  return sizeof(int) * 4 + (size_t)N * 2 * c.gam_cap * sizeof(double2) + N * sizeof(int) + (N + 1) * sizeof(int) +
         N * sizeof(int) + (size_t)(N + 1) * c.chi_cap * sizeof(double) + sizeof(double);
}
}  // namespace

pt_tebd_status pt_tebd_snapshot(pt_tebd_t h, void* buf, size_t* bytes) {
  if (!h || !bytes) return PT_TEBD_EINVAL;
  const ChainDev& M = h->chain_host[0];
  const int N = h->n_sites;
  const Caps& c = h->cap;
  const size_t need = snapshot_bytes(h);
  if (!buf) { *bytes = need; return PT_TEBD_OK; }
  if (*bytes < need) { *bytes = need; return PT_TEBD_ENOMEM; }
  char* p = static_cast<char*>(buf);
  int hdr[4] = {0x50545442, N, (int)c.gam_cap, h->step};
  std::memcpy(p, hdr, sizeof(hdr));
  p += sizeof(hdr);
  bool ok = true;
  auto d2h = [&](void* dev, size_t len) {
    ok = ok && check(hipMemcpyAsync(p, dev, len, hipMemcpyDeviceToHost, h->stream), h, "snapshot");
    p += len;
  };
  d2h(M.gam, (size_t)N * 2 * c.gam_cap * sizeof(double2));
  d2h(M.parity, N * sizeof(int));
  d2h(M.chi, (N + 1) * sizeof(int));
  d2h(M.xi, N * sizeof(int));
  d2h(M.lam, (size_t)(N + 1) * c.chi_cap * sizeof(double));
  d2h(M.log_scale, sizeof(double));
  if (!ok || !check(hipStreamSynchronize(h->stream), h, "sync")) return PT_TEBD_EDEVICE;
  *bytes = need;
  return device_status(h, 0);
}

pt_tebd_status pt_tebd_restore(pt_tebd_t h, const void* buf, size_t bytes) {
  if (!h || !buf) return PT_TEBD_EINVAL;
  const ChainDev& M = h->chain_host[0];
  const int N = h->n_sites;
  const Caps& c = h->cap;
  const char* p = static_cast<const char*>(buf);
  int hdr[4];
  if (bytes < snapshot_bytes(h)) { h->err = "snapshot buffer shorter than a snapshot of this handle"; return PT_TEBD_EINVAL; }
  std::memcpy(hdr, p, sizeof(hdr));
  if (hdr[0] != 0x50545442 || hdr[1] != N || hdr[2] != (int)c.gam_cap) { h->err = "snapshot does not match handle"; return PT_TEBD_EINVAL; }
  if (hdr[3] < 0 || (h->n_baths > 0 && hdr[3] > h->pt_steps)) { h->err = "snapshot step outside the PT-MPO range"; return PT_TEBD_EINVAL; }
  p += sizeof(hdr);
  bool ok = true;
  auto h2d = [&](void* dev, size_t len) {
    ok = ok && check(hipMemcpyAsync(dev, p, len, hipMemcpyHostToDevice, h->stream), h, "restore");
    p += len;
  };
  h2d(M.gam, (size_t)N * 2 * c.gam_cap * sizeof(double2));
  h2d(M.parity, N * sizeof(int));
  h2d(M.chi, (N + 1) * sizeof(int));
  h2d(M.xi, N * sizeof(int));
  h2d(M.lam, (size_t)(N + 1) * c.chi_cap * sizeof(double));
  h2d(M.log_scale, sizeof(double));
  const int zero = 0;  // a restored state carries no error of the state it replaces
  ok = ok && check(hipMemcpyAsync(M.status, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream), h, "restore");
  if (!ok || !check(hipStreamSynchronize(h->stream), h, "sync")) return PT_TEBD_EDEVICE;
  h->step = hdr[3];
  return PT_TEBD_OK;
}

int32_t pt_tebd_current_step(pt_tebd_t h) { return h ? h->step : -1; }

const char* pt_tebd_last_error(pt_tebd_t h) {
  if (h) return h->err.c_str();
  return t_create_error.empty() ? "null handle" : t_create_error.c_str();
}

void pt_tebd_destroy(pt_tebd_t h) {
  if (!h) return;
  hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->events) hipEventDestroy(e);
  delete h;
}

pt_tebd_status pt_tebd_step_many(pt_tebd_t* hs, int32_t n, int32_t n_steps) {
  if (!hs || n < 0 || n_steps < 0) return PT_TEBD_EINVAL;
  if (n == 0 || n_steps == 0) return PT_TEBD_OK;
  // a transient batch in memory of its own (pt_tebd_batch_* keeps one)
  size_t bytes = 0;
  pt_tebd_status s = pt_tebd_batch_workspace_size(hs, n, &bytes);
  if (s != PT_TEBD_OK) return s;
  void* ws = nullptr;
  if (hipMalloc(&ws, bytes) != hipSuccess) return PT_TEBD_ENOMEM;
  pt_tebd_batch_t b = nullptr;
  s = pt_tebd_batch_create(hs, n, ws, bytes, &b);
  if (s == PT_TEBD_OK) s = pt_tebd_batch_step(b, n_steps);
  if (b) pt_tebd_batch_destroy(b);  // synchronises the stream
  (void)hipFree(ws);
  return s;
}

pt_tebd_status pt_tebd_kernel_timing(pt_tebd_t h, int32_t kernel_class) {
  if (!h || kernel_class < KT_NONE || kernel_class > KT_BOND_GEMM) return PT_TEBD_EINVAL;
  if (!check(hipStreamSynchronize(h->stream), h, "sync")) return PT_TEBD_EDEVICE;
  h->timing_class = kernel_class;
  h->events_used = 0;
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  if (!check(hipMemcpy(h->timing_flops, zero, sizeof(zero), hipMemcpyHostToDevice), h, "timing reset"))
    return PT_TEBD_EDEVICE;
  return PT_TEBD_OK;
}

pt_tebd_status pt_tebd_kernel_timing_read(pt_tebd_t h, double* total_ms, int64_t* launches, double* alg_flops) {
  if (!h || !total_ms || !launches || !alg_flops) return PT_TEBD_EINVAL;
  if (!check(hipStreamSynchronize(h->stream), h, "sync")) return PT_TEBD_EDEVICE;
  double ms = 0.0;
  for (size_t i = 0; i + 1 < h->events_used; i += 2) {
    float t = 0.0f;
    if (!check(hipEventElapsedTime(&t, h->events[i], h->events[i + 1]), h, "event time")) return PT_TEBD_EDEVICE;
    ms += t;
  }
  double fl[4];
  if (!check(hipMemcpy(fl, h->timing_flops, sizeof(fl), hipMemcpyDeviceToHost), h, "timing read"))
    return PT_TEBD_EDEVICE;
  *total_ms = ms;
  *launches = (int64_t)(h->events_used / 2);
  *alg_flops = fl[0];
  return PT_TEBD_OK;
}

pt_tebd_status pt_tebd_gate(pt_tebd_t h, int32_t bond, double* out) {
  if (!h || !out || bond < 0 || bond >= (int)h->gates_host.size()) return PT_TEBD_EINVAL;
  const auto& g = h->gates_host[bond];
  for (size_t i = 0; i < g.size(); ++i) {
    out[2 * i] = g[i].real();
    out[2 * i + 1] = g[i].imag();
  }
  return PT_TEBD_OK;
}

pt_tebd_status pt_bath_eta(double alpha, double wc, int32_t cutoff_kind, double temperature, double dt,
                           int32_t mem_steps, double* eta_out) {
  if (!eta_out) return PT_TEBD_EINVAL;
  std::vector<cplx> eta;
  std::string err;
  if (!ptt::bath_eta(alpha, wc, cutoff_kind, temperature, dt, mem_steps, eta, err)) return PT_TEBD_EINVAL;
  for (size_t i = 0; i < eta.size(); ++i) {
    eta_out[2 * i] = eta[i].real();
    eta_out[2 * i + 1] = eta[i].imag();
  }
  return PT_TEBD_OK;
}

pt_tebd_status pt_mpo_build_ohmic(double alpha, double wc, int32_t cutoff_kind, double temperature, double dt,
                                  int32_t n_steps, int32_t mem_steps, double eps, int32_t xi_max,
                                  const double* coupling_op, int32_t d, pt_tebd_bath* out) {
  if (!out || !coupling_op || d != 2 || n_steps < 1 || mem_steps < 0 || xi_max < 1 || !(eps >= 0.0))
    return PT_TEBD_EINVAL;
  std::vector<cplx> eta;
  std::string err;
  if (!ptt::bath_eta(alpha, wc, cutoff_kind, temperature, dt, mem_steps, eta, err)) return PT_TEBD_EINVAL;
  // coupling eigenbasis: keep the computational basis when diagonal
  cplx s[4];
  for (int i = 0; i < 4; ++i) s[i] = {coupling_op[2 * i], coupling_op[2 * i + 1]};
  if (std::abs(s[1] - std::conj(s[2])) > 1e-12 || std::abs(s[0].imag()) > 1e-12 || std::abs(s[3].imag()) > 1e-12)
    return PT_TEBD_EINVAL;
  const bool diag = std::abs(s[1]) == 0.0 && std::abs(s[2]) == 0.0;
  std::vector<double> sigma(2);
  std::vector<cplx> u(4, 0.0);
  if (diag) {
    sigma = {s[0].real(), s[3].real()};
    u[0] = u[3] = 1.0;
  } else {
    double w[2];
    ptt::heev(2, s, w, u.data());
    sigma = {w[0], w[1]};
  }
  std::vector<std::vector<cplx>> tens;
  std::vector<int> dims;
  if (!ptt::build_ptmpo(eta, sigma, n_steps, eps, xi_max, tens, dims, err)) return PT_TEBD_EINVAL;
  out->site = 0;
  out->n_steps = n_steps;
  out->diagonal = diag ? 1 : 0;
  int32_t* bd = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (n_steps + 1)));
  const double** tp = static_cast<const double**>(std::malloc(sizeof(double*) * n_steps));
  if (!bd || !tp) return PT_TEBD_ENOMEM;
  for (int k = 0; k <= n_steps; ++k) bd[k] = dims[k];
  // W = U kron conj(U): eigenbasis vec -> computational vec
  cplx wmat[16];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) wmat[(i * 2 + j) * 4 + (k * 2 + l)] = u[i * 2 + k] * std::conj(u[j * 2 + l]);
  for (int k = 0; k < n_steps; ++k) {
    const int xa = dims[k], xb = dims[k + 1];
    const size_t per = diag ? 4 : 16;
    double* t = static_cast<double*>(std::malloc(sizeof(double) * 2 * per * xa * xb));
    if (!t) return PT_TEBD_ENOMEM;
    for (int e = 0; e < xa; ++e)
      for (int f = 0; f < xb; ++f) {
        const cplx* p = &tens[k][((size_t)e * xb + f) * 4];
        if (diag) {
          for (int x = 0; x < 4; ++x) {
            t[2 * (((size_t)e * xb + f) * 4 + x)] = p[x].real();
            t[2 * (((size_t)e * xb + f) * 4 + x) + 1] = p[x].imag();
          }
        } else {
          for (int so = 0; so < 4; ++so)
            for (int si = 0; si < 4; ++si) {
              cplx acc = 0.0;
              for (int x = 0; x < 4; ++x) acc += wmat[so * 4 + x] * p[x] * std::conj(wmat[si * 4 + x]);
              const size_t q = (((size_t)e * xb + f) * 4 + so) * 4 + si;
              t[2 * q] = acc.real();
              t[2 * q + 1] = acc.imag();
            }
        }
      }
    tp[k] = t;
  }
  out->bond_dims = bd;
  out->tensors = tp;
  out->caps = nullptr;
  out->initial = nullptr;
  return PT_TEBD_OK;
}

void pt_mpo_free(pt_tebd_bath* b) {
  if (!b) return;
  if (b->tensors)
    for (int k = 0; k < b->n_steps; ++k) std::free(const_cast<double*>(b->tensors[k]));
  std::free(const_cast<double**>(b->tensors));
  std::free(const_cast<int32_t*>(b->bond_dims));
  b->tensors = nullptr;
  b->bond_dims = nullptr;
}

}  // extern "C"

// ================================================================== batch
// Many chains advanced together: every kernel of a sublayer runs once over
// the bond updates of all chains (the job tables of the chains
// concatenated), the PT absorption once over all (chain, bath) pairs, and a
// device step counter per chain keeps the launch sequence identical from
// step to step, so one step is captured in a HIP graph and replayed.
struct pt_tebd_batch {
  std::vector<pt_tebd*> hs;
  hipStream_t stream = nullptr;
  Exec x{};
  Sublayer sub[2];                 // [0] even bonds (1-based), [1] odd bonds
  ChainDev* chains = nullptr;      // device [n]
  ptt::BathRef* refs = nullptr;    // device [n_refs]
  int n_refs = 0;
  int* kstep = nullptr;            // device [n]
  std::vector<int> kstep_host;
  int mixed = 0, gemm_valu = 0;
  unsigned mixed_mask = ~(1u << 30);
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string err;
};

namespace {

struct BatchPtrs {
  ChainDev* chains;
  int* kstep;
  ptt::BathRef* refs;
  BondJob* jobs[2];
  HeevJob *hb[2], *hoy[2], *hoz[2], *hoyb[2], *hozb[2], *hl2[2], *hl2b[2], *hrr[2], *hrb[2], *hrd[2];
  ptt::RefineJob *rb[2], *rd[2];
};

size_t batch_layout(int n, const int tot[2], int n_refs, void* base, BatchPtrs* out) {
  Bump bp(base);
  BatchPtrs P{};
  P.chains = bp.take<ChainDev>(n);
  P.kstep = bp.take<int>(n);
  P.refs = bp.take<ptt::BathRef>(std::max(n_refs, 1));
  for (int par = 0; par < 2; ++par) {
    const int t = std::max(tot[par], 1);
    P.jobs[par] = bp.take<BondJob>(t);
    P.hb[par] = bp.take<HeevJob>(2 * t);
    P.hoy[par] = bp.take<HeevJob>(t);
    P.hoz[par] = bp.take<HeevJob>(t);
    P.hoyb[par] = bp.take<HeevJob>(t);
    P.hozb[par] = bp.take<HeevJob>(t);
    P.hl2[par] = bp.take<HeevJob>(t);
    P.hl2b[par] = bp.take<HeevJob>(t);
    P.hrr[par] = bp.take<HeevJob>(t);
    P.hrb[par] = bp.take<HeevJob>(2 * t);
    P.hrd[par] = bp.take<HeevJob>(t);
    P.rb[par] = bp.take<ptt::RefineJob>(2 * t);
    P.rd[par] = bp.take<ptt::RefineJob>(t);
  }
  if (out) *out = P;
  return bp.off + 256;
}

pt_tebd_status batch_check(pt_tebd_t* hs, int n, std::string& err) {
  if (!hs || n < 1) { err = "empty batch"; return PT_TEBD_EINVAL; }
  for (int i = 0; i < n; ++i) {
    const pt_tebd* h = hs[i];
    if (!h) { err = "null handle in batch"; return PT_TEBD_EINVAL; }
    for (int j = 0; j < i; ++j)
      if (hs[j] == h) { err = "a handle appears twice in the batch"; return PT_TEBD_EINVAL; }
    if (h->n_sites < 2) { err = "batched chains need at least two sites"; return PT_TEBD_EINVAL; }
    const pt_tebd* f = hs[0];
    if (h->stream != f->stream) { err = "batched handles must share one stream"; return PT_TEBD_EINVAL; }
    if (h->precision != f->precision || h->gemm_valu != f->gemm_valu || h->mixed_mask != f->mixed_mask) {
      err = "batched handles must share the precision";
      return PT_TEBD_EINVAL;
    }
    if (h->power_iters != f->power_iters || h->cholqr != f->cholqr || h->deflate != f->deflate ||
        h->refine_levels != f->refine_levels || h->refine_tau != f->refine_tau) {
      err = "batched handles must share the range finder and refinement settings";
      return PT_TEBD_EINVAL;
    }
  }
  return PT_TEBD_OK;
}

void batch_counts(pt_tebd_t* hs, int n, int tot[2], int& n_refs) {
  tot[0] = tot[1] = 0;
  n_refs = 0;
  for (int i = 0; i < n; ++i) {
    tot[0] += (int)hs[i]->sub_even.bonds.size();
    tot[1] += (int)hs[i]->sub_odd.bonds.size();
    n_refs += hs[i]->n_baths;
  }
}

void batch_enqueue_step(pt_tebd_batch* b) {
  const Exec& x = b->x;
  auto half = [&]() {
    run_sublayer(x, b->sub[0], b->chains);
    run_sublayer(x, b->sub[1], b->chains);
    run_sublayer(x, b->sub[0], b->chains);
  };
  half();
  if (b->n_refs > 0) {
    ptt::k_pt_absorb_batch<<<dim3(elem_blocks((long long)x.cap.chi_cap * 4 * x.cap.xi_cap * x.cap.chi_cap),
                                  b->n_refs), kThreads, 0, x.stream>>>(b->chains, b->refs, b->kstep);
    ptt::k_pt_commit_batch<<<(b->n_refs + 63) / 64, 64, 0, x.stream>>>(b->chains, b->refs, b->n_refs, b->kstep);
  }
  half();
  const int n = (int)b->hs.size();
  ptt::k_advance_steps<<<(n + 63) / 64, 64, 0, x.stream>>>(b->kstep, n);
}

// the GEMM engine flags of the batch's precision while its steps are enqueued
struct BatchScope {
  int pm, pv;
  unsigned pk;
  pt_tebd* pt;
  explicit BatchScope(const pt_tebd_batch* b)
      : pm(t_gemm_mixed), pv(t_gemm_valu), pk(t_gemm_mixed_mask), pt(t_timing) {
    t_gemm_mixed = b->mixed;
    t_gemm_valu = b->gemm_valu;
    t_gemm_mixed_mask = b->mixed_mask;
    t_timing = nullptr;
  }
  ~BatchScope() {
    t_gemm_mixed = pm;
    t_gemm_valu = pv;
    t_gemm_mixed_mask = pk;
    t_timing = pt;
  }
};

}  // namespace

extern "C" pt_tebd_status pt_tebd_batch_workspace_size(pt_tebd_t* hs, int32_t n, size_t* bytes) {
  std::string err;
  if (!bytes) return PT_TEBD_EINVAL;
  const pt_tebd_status s = batch_check(hs, n, err);
  if (s != PT_TEBD_OK) return s;
  int tot[2], n_refs;
  batch_counts(hs, n, tot, n_refs);
  *bytes = batch_layout(n, tot, n_refs, nullptr, nullptr);
  return PT_TEBD_OK;
}

extern "C" pt_tebd_status pt_tebd_batch_create(pt_tebd_t* hs, int32_t n, void* ws, size_t bytes,
                                               pt_tebd_batch_t* out) {
  if (!out) return PT_TEBD_EINVAL;
  *out = nullptr;
  std::string err;
  pt_tebd_status s = batch_check(hs, n, err);
  if (s != PT_TEBD_OK) { t_create_error = err; return s; }
  int tot[2], n_refs;
  batch_counts(hs, n, tot, n_refs);
  const size_t need = batch_layout(n, tot, n_refs, nullptr, nullptr);
  if (!ws || bytes < need) { t_create_error = "batch workspace smaller than pt_tebd_batch_workspace_size"; return PT_TEBD_ENOMEM; }
  BatchPtrs P;
  batch_layout(n, tot, n_refs, ws, &P);
  auto b = std::make_unique<pt_tebd_batch>();
  b->hs.assign(hs, hs + n);
  const pt_tebd* f = hs[0];
  b->stream = f->stream;
  b->mixed = f->precision == PT_TEBD_FP32_MIXED ? 1 : 0;
  b->gemm_valu = f->gemm_valu;
  b->mixed_mask = f->mixed_mask;
  b->use_graph = env_int("PT_TEBD_GRAPH", 1) != 0 && b->stream != nullptr;
  Caps c = f->cap;
  for (int i = 1; i < n; ++i) {
    const Caps& d = hs[i]->cap;
    c.chi_cap = std::max(c.chi_cap, d.chi_cap); c.xi_cap = std::max(c.xi_cap, d.xi_cap);
    c.nb = std::max(c.nb, d.nb); c.dn = std::max(c.dn, d.dn); c.kc = std::max(c.kc, d.kc);
    c.ks = std::max(c.ks, d.ks); c.nh = std::max(c.nh, d.nh); c.gam_cap = std::max(c.gam_cap, d.gam_cap);
  }
  b->x = Exec{b->stream, c, f->power_iters, f->cholqr, f->deflate, f->refine_levels, f->refine_tau};
  hipStream_t st = b->stream;
  bool ok = true;
  auto cp = [&](void* dst, const void* src, size_t len, hipMemcpyKind kind) {
    ok = ok && hipMemcpyAsync(dst, src, len, kind, st) == hipSuccess;
  };
  std::vector<ChainDev> ch(n);
  std::vector<ptt::BathRef> refs;
  for (int i = 0; i < n; ++i) {
    ch[i] = hs[i]->chain_host[0];
    for (int j = 0; j < hs[i]->n_baths; ++j) refs.push_back(ptt::BathRef{i, 0, hs[i]->baths + j});
  }
  cp(P.chains, ch.data(), n * sizeof(ChainDev), hipMemcpyHostToDevice);
  if (n_refs) cp(P.refs, refs.data(), n_refs * sizeof(ptt::BathRef), hipMemcpyHostToDevice);
  b->n_refs = n_refs;
  for (int par = 0; par < 2; ++par) {
    Sublayer& S = b->sub[par];
    S.jobs = P.jobs[par]; S.heev_b = P.hb[par]; S.heev_oy = P.hoy[par]; S.heev_oz = P.hoz[par];
    S.heev_oyb = P.hoyb[par]; S.heev_ozb = P.hozb[par]; S.heev_l2 = P.hl2[par]; S.heev_l2b = P.hl2b[par];
    S.heev_rr = P.hrr[par]; S.ref_b = P.rb[par]; S.ref_d = P.rd[par]; S.heev_ref_b = P.hrb[par];
    S.heev_ref_d = P.hrd[par];
    int off = 0;
    for (int i = 0; i < n; ++i) {
      const Sublayer& H = par == 0 ? hs[i]->sub_even : hs[i]->sub_odd;
      const int m = (int)H.bonds.size();
      if (m == 0) continue;
      for (int j = 0; j < m; ++j) {
        BondJob J = H.host_jobs[j];
        J.chain = i;
        S.host_jobs.push_back(J);
        S.bonds.push_back(H.bonds[j]);
      }
      auto d2d = [&](void* dst_base, const void* src, size_t per, int count) {
        cp(static_cast<char*>(dst_base) + per * (size_t)off * (count / m), src, per * count, hipMemcpyDeviceToDevice);
      };
      d2d(S.heev_b, H.heev_b, sizeof(HeevJob), 2 * m);
      d2d(S.heev_oy, H.heev_oy, sizeof(HeevJob), m);
      d2d(S.heev_oz, H.heev_oz, sizeof(HeevJob), m);
      d2d(S.heev_oyb, H.heev_oyb, sizeof(HeevJob), m);
      d2d(S.heev_ozb, H.heev_ozb, sizeof(HeevJob), m);
      d2d(S.heev_l2, H.heev_l2, sizeof(HeevJob), m);
      d2d(S.heev_l2b, H.heev_l2b, sizeof(HeevJob), m);
      d2d(S.heev_rr, H.heev_rr, sizeof(HeevJob), m);
      d2d(S.heev_ref_b, H.heev_ref_b, sizeof(HeevJob), 2 * m);
      d2d(S.heev_ref_d, H.heev_ref_d, sizeof(HeevJob), m);
      d2d(S.ref_b, H.ref_b, sizeof(ptt::RefineJob), 2 * m);
      d2d(S.ref_d, H.ref_d, sizeof(ptt::RefineJob), m);
      off += m;
    }
    if (!S.host_jobs.empty()) cp(S.jobs, S.host_jobs.data(), S.host_jobs.size() * sizeof(BondJob), hipMemcpyHostToDevice);
  }
  b->chains = P.chains;
  b->refs = P.refs;
  b->kstep = P.kstep;
  b->kstep_host.assign(n, 0);
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) { t_create_error = "batch set-up copies failed"; return PT_TEBD_EDEVICE; }
  *out = b.release();
  return PT_TEBD_OK;
}

extern "C" pt_tebd_status pt_tebd_batch_step(pt_tebd_batch_t b, int32_t n_steps) {
  if (!b || n_steps < 0) return PT_TEBD_EINVAL;
  for (pt_tebd* h : b->hs)
    if (h->n_baths > 0 && h->step + n_steps > h->pt_steps) {
      b->err = "stepping past the end of a PT-MPO";
      return PT_TEBD_ERANGE;
    }
  if (n_steps == 0) return PT_TEBD_OK;
  BatchScope scope(b);
  hipStream_t st = b->stream;
  for (size_t i = 0; i < b->hs.size(); ++i) b->kstep_host[i] = b->hs[i]->step;
  if (hipMemcpyAsync(b->kstep, b->kstep_host.data(), b->hs.size() * sizeof(int), hipMemcpyHostToDevice, st) !=
      hipSuccess) { b->err = "step counter upload"; return PT_TEBD_EDEVICE; }
  if (b->use_graph) {
    if (!b->gexec) {
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        b->err = "graph capture could not start";
        return PT_TEBD_EDEVICE;
      }
      batch_enqueue_step(b);
      if (hipStreamEndCapture(st, &b->graph) != hipSuccess ||
          hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
        b->err = "graph capture or instantiation failed";
        return PT_TEBD_EDEVICE;
      }
    }
    for (int k = 0; k < n_steps; ++k)
      if (hipGraphLaunch(b->gexec, st) != hipSuccess) { b->err = "graph launch"; return PT_TEBD_EDEVICE; }
  } else {
    for (int k = 0; k < n_steps; ++k) batch_enqueue_step(b);
  }
  if (hipGetLastError() != hipSuccess) { b->err = "kernel launch"; return PT_TEBD_EDEVICE; }
  for (pt_tebd* h : b->hs) h->step += n_steps;
  return PT_TEBD_OK;
}

extern "C" const char* pt_tebd_batch_last_error(pt_tebd_batch_t b) {
  if (b) return b->err.c_str();
  return t_create_error.empty() ? "null batch" : t_create_error.c_str();
}

extern "C" void pt_tebd_batch_destroy(pt_tebd_batch_t b) {
  if (!b) return;
  hipStreamSynchronize(b->stream);
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->graph) hipGraphDestroy(b->graph);
  delete b;
}

// ================================================= PT-MPO builds on the GPU
namespace {
// coupling eigenbasis of a d = 2 Hermitian operator: eigenvalues, the
// eigenvector matrix, and whether the operator is already diagonal
bool coupling_basis(const double* op, std::vector<double>& sigma, std::vector<cplx>& u, bool& diag) {
  cplx s[4];
  for (int i = 0; i < 4; ++i) s[i] = {op[2 * i], op[2 * i + 1]};
  if (std::abs(s[1] - std::conj(s[2])) > 1e-12 || std::abs(s[0].imag()) > 1e-12 || std::abs(s[3].imag()) > 1e-12)
    return false;
  diag = std::abs(s[1]) == 0.0 && std::abs(s[2]) == 0.0;
  u.assign(4, 0.0);
  if (diag) {
    sigma = {s[0].real(), s[3].real()};
    u[0] = u[3] = 1.0;
  } else {
    double w[2];
    ptt::heev(2, s, w, u.data());
    sigma = {w[0], w[1]};
  }
  return true;
}

// P_k in the coupling eigenbasis ([e][e'][x]) -> the bath struct's layout:
// unchanged when the coupling is diagonal, else W P W^-1 with W = U (x) U*
// on the Liouville index ([e][e'][s_out][s_in])
void fill_bath(int n_steps, const std::vector<int>& dims, const std::vector<std::vector<cplx>>& tens, bool diag,
               const std::vector<cplx>& u, pt_tebd_bath* out) {
  out->site = 0;
  out->n_steps = n_steps;
  out->diagonal = diag ? 1 : 0;
  int32_t* bd = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (n_steps + 1)));
  const double** tp = static_cast<const double**>(std::malloc(sizeof(double*) * n_steps));
  for (int k = 0; k <= n_steps; ++k) bd[k] = dims[k];
  cplx wmat[16];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) wmat[(i * 2 + j) * 4 + (k * 2 + l)] = u[i * 2 + k] * std::conj(u[j * 2 + l]);
  for (int k = 0; k < n_steps; ++k) {
    const int xa = dims[k], xb = dims[k + 1];
    const size_t per = diag ? 4 : 16;
    double* t = static_cast<double*>(std::malloc(sizeof(double) * 2 * per * xa * xb));
    for (int e = 0; e < xa; ++e)
      for (int f = 0; f < xb; ++f) {
        const cplx* p = &tens[k][((size_t)e * xb + f) * 4];
        if (diag) {
          for (int x = 0; x < 4; ++x) {
            t[2 * (((size_t)e * xb + f) * 4 + x)] = p[x].real();
            t[2 * (((size_t)e * xb + f) * 4 + x) + 1] = p[x].imag();
          }
        } else {
          for (int so = 0; so < 4; ++so)
            for (int si = 0; si < 4; ++si) {
              cplx acc = 0.0;
              for (int x = 0; x < 4; ++x) acc += wmat[so * 4 + x] * p[x] * std::conj(wmat[si * 4 + x]);
              const size_t q = (((size_t)e * xb + f) * 4 + so) * 4 + si;
              t[2 * q] = acc.real();
              t[2 * q + 1] = acc.imag();
            }
        }
      }
    tp[k] = t;
  }
  out->bond_dims = bd;
  out->tensors = tp;
  out->caps = nullptr;
  out->initial = nullptr;
}
}  // namespace

extern "C" pt_tebd_status pt_mpo_build_ohmic_batch(int32_t n_builds, const pt_bath_params* params, double dt,
                                                   int32_t n_steps, int32_t mem_steps, double eps, int32_t xi_max,
                                                   int32_t d, void* hip_stream, pt_tebd_bath* out) {
  if (n_builds < 1 || !params || !out || d != 2 || n_steps < 1 || mem_steps < 0 || xi_max < 1 || xi_max > 256 ||
      !(eps >= 0.0) || !(dt > 0.0))
    return PT_TEBD_EINVAL;
  const int K = mem_steps, M = n_steps, acap = 4 * xi_max;
  const size_t slot = (size_t)acap * 4 * acap;
  std::vector<std::vector<double>> sigmas(n_builds);
  std::vector<std::vector<cplx>> us(n_builds);
  std::vector<char> diag(n_builds);
  std::vector<double2> bfac((size_t)n_builds * (K + 1) * 16);
  std::vector<int> len(n_builds);
  for (int b = 0; b < n_builds; ++b) {
    const pt_bath_params& P = params[b];
    if (!P.coupling_op || P.n_steps < 0 || P.n_steps > n_steps) return PT_TEBD_EINVAL;
    len[b] = P.n_steps > 0 ? P.n_steps : n_steps;
    bool dg = false;
    if (!coupling_basis(P.coupling_op, sigmas[b], us[b], dg)) return PT_TEBD_EINVAL;
    diag[b] = dg;
    std::vector<cplx> eta;
    std::string err;
    if (!ptt::bath_eta(P.alpha, P.wc, P.cutoff_kind, P.temperature, dt, K, eta, err)) return PT_TEBD_EINVAL;
    const std::vector<double>& sg = sigmas[b];
    for (int dl = 0; dl <= K; ++dl)
      for (int x = 0; x < 4; ++x)
        for (int xp = 0; xp < 4; ++xp) {
          const double spx = sg[x / 2], smx = sg[x % 2], spy = sg[xp / 2], smy = sg[xp % 2];
          const cplx v = std::exp(-(spx - smx) * (eta[dl] * spy - std::conj(eta[dl]) * smy));
          bfac[((size_t)b * (K + 1) + dl) * 16 + x * 4 + xp] = ptt::mk<double>(v.real(), v.imag());
        }
  }
  // device memory of the builds (a host helper, not the per-step path)
  Bump sz(nullptr);
  // per build: the stage jobs, their eigensolver jobs, and the refinement of
  // small singular values (rows of W^H M right to left, columns of M W left
  // to right) with its own eigensolver jobs
  struct Dev {
    double2* bf;
    ptt::TempoJob* jobs;
    HeevJob *hrl, *hlr, *hrl_ref, *hlr_ref;
    ptt::RefineJob *rrl, *rlr;
  };
  struct Host {
    std::vector<ptt::TempoJob> jobs;
    std::vector<HeevJob> hrl, hlr, hrl_ref, hlr_ref;
    std::vector<ptt::RefineJob> rrl, rlr;
  };
  auto plan = [&](Bump& bp, Host* h, Dev& dv) {
    dv.bf = bp.take<double2>(bfac.size());
    dv.jobs = bp.take<ptt::TempoJob>(n_builds);
    dv.hrl = bp.take<HeevJob>(n_builds);
    dv.hlr = bp.take<HeevJob>(n_builds);
    dv.hrl_ref = bp.take<HeevJob>(n_builds);
    dv.hlr_ref = bp.take<HeevJob>(n_builds);
    dv.rrl = bp.take<ptt::RefineJob>(n_builds);
    dv.rlr = bp.take<ptt::RefineJob>(n_builds);
    for (int b = 0; b < n_builds; ++b) {
      ptt::TempoJob J{};
      J.K = K; J.M = len[b]; J.xi_cap = xi_max; J.acap = acap; J.eps = eps;
      J.bfac = dv.bf ? dv.bf + (size_t)b * (K + 1) * 16 : nullptr;
      J.slots = bp.take<double2>((size_t)(K + 1) * slot);
      J.sa = bp.take<int>(K + 1);
      J.sc = bp.take<int>(K + 1);
      J.tmp = bp.take<double2>(slot);
      J.g = bp.take<double2>((size_t)acap * acap);
      J.w = bp.take<double2>((size_t)acap * acap);
      J.p = bp.take<double2>((size_t)4 * acap * acap);
      J.lam = bp.take<double>(acap);
      J.s = bp.take<double>(acap);
      J.perm = bp.take<int>(acap);
      J.sd = bp.take<int>(ptt::TS_COUNT);
      J.out = bp.take<double2>((size_t)M * xi_max * xi_max * 4);
      J.out_dims = bp.take<int>(M + 1);
      J.status = bp.take<int>(1);
      double2* refl = bp.take<double2>((size_t)acap * acap);
      double* tri = bp.take<double>(6 * (size_t)acap);
      double* work = bp.take<double>(8 * (size_t)acap * acap);
      double* z = bp.take<double>((size_t)acap * acap);
      double2* rw = bp.take<double2>((size_t)acap * acap);     // block eigenvectors
      double2* tp = bp.take<double2>((size_t)4 * acap * acap); // rotated block of p
      double2* tv = bp.take<double2>((size_t)acap * acap);     // rotated block of w
      int* blk = bp.take<int>(4);
      if (h) {
        h->jobs.push_back(J);
        HeevJob H{};
        H.a = J.g; H.lda = acap; H.n_ptr = J.sd + ptt::TS_N; H.w = J.lam; H.refl = refl; H.tri = tri;
        H.work = work; H.z = z; H.n_cap = acap; H.nvec_out = J.sd + ptt::TS_KEEP; H.rule = ptt::RULE_FULL;
        H.eps = 0.0; H.cap = 0; H.extra_tail = nullptr; H.rank_tol = 0.0; H.v = J.w; H.ldv = acap;
        H.scale = ptt::SCALE_NONE; H.status = J.status; H.noise_cluster = 1; H.abs_ref = nullptr; H.abs_tol = 0.0;
        h->hrl.push_back(H);
        H.rule = ptt::RULE_FULL;
        h->hlr.push_back(H);
        // the block Gram matrix goes into g (free between the projection and
        // the finishing kernels), its eigenvectors into rw
        HeevJob HR = H;
        HR.n_ptr = blk + 1; HR.nvec_out = blk + 2; HR.v = rw; HR.rule = ptt::RULE_FULL;
        h->hrl_ref.push_back(HR);
        h->hlr_ref.push_back(HR);
        ptt::RefineJob R{};
        R.blk = blk; R.G = J.g; R.ldg = acap; R.W = rw; R.ldw = acap; R.TP = tp; R.TV = tv; R.ldtv = acap;
        R.V = J.w; R.ldv = acap; R.s = J.s; R.P = J.p; R.ldp_ptr = J.sd + ptt::TS_COLS;
        R.len_cols = J.sd + ptt::TS_ROWS; R.len_rows = J.sd + ptt::TS_COLS;
        // right to left: the keep rows of p = W^H M (a x (d^2 c)); W is a x keep
        ptt::RefineJob RL = R;
        RL.cols = 0; RL.n_ptr = J.sd + ptt::TS_KEEP; RL.nv_ptr = J.sd + ptt::TS_ROWS; RL.ldtp = 4 * acap;
        h->rrl.push_back(RL);
        // left to right: the columns of p = M W ((a d^2) x c); W is c x c
        ptt::RefineJob LR = R;
        LR.cols = 1; LR.n_ptr = J.sd + ptt::TS_COLS; LR.nv_ptr = J.sd + ptt::TS_COLS; LR.ldtp = acap;
        h->rlr.push_back(LR);
      }
    }
  };
  Dev dv{};
  plan(sz, nullptr, dv);
  const size_t bytes = sz.off + 256;
  void* ws = nullptr;
  if (hipMalloc(&ws, bytes) != hipSuccess) return PT_TEBD_ENOMEM;
  Bump bp(ws);
  Host hs;
  plan(bp, &hs, dv);
  std::vector<ptt::TempoJob>& jobs = hs.jobs;
  ptt::TempoJob* jobs_dev = dv.jobs;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  auto up = [&](void* dst, const void* src, size_t b) {
    return hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = up(dv.bf, bfac.data(), bfac.size() * sizeof(double2)) &&
            up(dv.jobs, jobs.data(), n_builds * sizeof(ptt::TempoJob)) &&
            up(dv.hrl, hs.hrl.data(), n_builds * sizeof(HeevJob)) && up(dv.hlr, hs.hlr.data(), n_builds * sizeof(HeevJob)) &&
            up(dv.hrl_ref, hs.hrl_ref.data(), n_builds * sizeof(HeevJob)) &&
            up(dv.hlr_ref, hs.hlr_ref.data(), n_builds * sizeof(HeevJob)) &&
            up(dv.rrl, hs.rrl.data(), n_builds * sizeof(ptt::RefineJob)) &&
            up(dv.rlr, hs.rlr.data(), n_builds * sizeof(ptt::RefineJob));
  // three levels of refinement, each resolving singular values four decades
  // further below the largest one than the level before
  Exec tx{};
  tx.stream = st;
  tx.refine_levels = 3;
  tx.refine_tau = 1e-4;
  for (int b = 0; b < n_builds && ok; ++b)
    ok = hipMemsetAsync(jobs[b].status, 0, sizeof(int), st) == hipSuccess;
  const int tiles = (4 * acap + ptt::GEMM_BM - 1) / ptt::GEMM_BM;
  const dim3 gg(tiles, tiles, n_builds);
  const int sb = (n_builds + 63) / 64;
  for (int k = 1; k <= M && ok; ++k) {
    ptt::k_tempo_begin<<<n_builds, 256, 0, st>>>(jobs_dev, k);
    const int m = std::min(K, k - 1);
    for (int i = 0; i < m; ++i) {  // right to left: site k - i = L Q
      ptt::k_tempo_stage<<<sb, 64, 0, st>>>(jobs_dev, n_builds, k, i, 1);
      ptt::k_tempo_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs_dev, ptt::TG_RL_GRAM);
      launch_heev(st, dv.hrl, n_builds, acap);
      ptt::k_tempo_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs_dev, ptt::TG_RL_PROJ);
      run_refine(tx, dv.rrl, dv.hrl_ref, n_builds, acap, 4 * acap, acap);
      ptt::k_tempo_rl_finish<<<n_builds, 256, 0, st>>>(jobs_dev);
      ptt::k_tempo_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs_dev, ptt::TG_RL_PUSH);
      ptt::k_tempo_push_copy<<<n_builds, 256, 0, st>>>(jobs_dev, 1);
    }
    for (int i = 0; i < m; ++i) {  // left to right: truncated SVD of site k - m + i
      ptt::k_tempo_stage<<<sb, 64, 0, st>>>(jobs_dev, n_builds, k, i, 0);
      ptt::k_tempo_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs_dev, ptt::TG_LR_GRAM);
      launch_heev(st, dv.hlr, n_builds, acap);
      ptt::k_tempo_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs_dev, ptt::TG_LR_PROJ);
      run_refine(tx, dv.rlr, dv.hlr_ref, n_builds, 4 * acap, acap, acap);
      ptt::k_tempo_lr_rule<<<n_builds, 256, 0, st>>>(jobs_dev);
      ptt::k_tempo_gemm<<<gg, ptt::GEMM_THREADS, 0, st>>>(jobs_dev, ptt::TG_LR_PUSH);
      ptt::k_tempo_push_copy<<<n_builds, 256, 0, st>>>(jobs_dev, 0);
    }
  }
  if (ok) ptt::k_tempo_end<<<n_builds, 256, 0, st>>>(jobs_dev);
  ok = ok && hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
  // results to the host
  for (int b = 0; b < n_builds && ok; ++b) {
    const int Mb = len[b];
    std::vector<int> dims(Mb + 1);
    int status = 0;
    std::vector<double2> o((size_t)Mb * xi_max * xi_max * 4);
    ok = hipMemcpy(dims.data(), jobs[b].out_dims, (Mb + 1) * sizeof(int), hipMemcpyDeviceToHost) == hipSuccess &&
         hipMemcpy(&status, jobs[b].status, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess &&
         hipMemcpy(o.data(), jobs[b].out, o.size() * sizeof(double2), hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) break;
    if (status & 4) { ok = false; break; }
    std::vector<std::vector<cplx>> tens(Mb);
    for (int k = 0; k < Mb; ++k) {
      const int xa = dims[k], xb = dims[k + 1];
      tens[k].resize((size_t)xa * xb * 4);
      for (size_t q = 0; q < tens[k].size(); ++q) {
        const double2 v = o[(size_t)k * xi_max * xi_max * 4 + q];
        tens[k][q] = {v.x, v.y};
      }
    }
    fill_bath(Mb, dims, tens, diag[b] != 0, us[b], &out[b]);
  }
  (void)hipFree(ws);
  return ok ? PT_TEBD_OK : PT_TEBD_EDEVICE;
}

// ------------------------------------------------------------ test hooks
#include "pt_tebd_testing.h"

namespace {
// pt_test_heev and pt_test_heev_tridiagonal: the eigensolver on one matrix;
// tri (2 n doubles: diagonal, off-diagonal of T) and z (n x n, the
// eigenvectors of T, row-major) are copied out when given
pt_tebd_status test_heev(int32_t n, const double* a, int32_t rule, double eps, int32_t cap, double* w, double* v,
                         int32_t* nvec, double* tri, double* z) {
  if (n < 1 || n > 1024 || !a || !w || !v || !nvec) return PT_TEBD_EINVAL;
  const size_t nn = (size_t)n * n;
  double2 *da = nullptr, *drefl = nullptr, *dv = nullptr;
  double *dw = nullptr, *dtri = nullptr, *dwork = nullptr, *dz = nullptr, *dextra = nullptr;
  int *dn = nullptr, *dnvec = nullptr, *dstat = nullptr;
  HeevJob* djob = nullptr;
  bool ok = hipMalloc(&da, nn * sizeof(double2)) == hipSuccess && hipMalloc(&drefl, nn * sizeof(double2)) == hipSuccess &&
            hipMalloc(&dv, nn * sizeof(double2)) == hipSuccess && hipMalloc(&dw, n * sizeof(double)) == hipSuccess &&
            hipMalloc(&dtri, 6 * n * sizeof(double)) == hipSuccess && hipMalloc(&dwork, 8 * nn * sizeof(double)) == hipSuccess &&
            hipMalloc(&dz, nn * sizeof(double)) == hipSuccess && hipMalloc(&dextra, sizeof(double)) == hipSuccess &&
            hipMalloc(&dn, sizeof(int)) == hipSuccess && hipMalloc(&dnvec, sizeof(int)) == hipSuccess &&
            hipMalloc(&dstat, sizeof(int)) == hipSuccess && hipMalloc(&djob, sizeof(HeevJob)) == hipSuccess;
  pt_tebd_status st = PT_TEBD_OK;
  if (ok) {
    HeevJob J{};
    const int r = rule == 0 ? ptt::RULE_ALL : rule == 1 ? ptt::RULE_EPS : rule == 2 ? ptt::RULE_CAP
                : rule == 3 ? ptt::RULE_RANK : ptt::RULE_FULL;
    fill_heev(J, da, n, dn, dw, drefl, dtri, dwork, dz, n, dnvec, r, eps, cap, dextra, eps, dv, n, ptt::SCALE_NONE, dstat);
    const double zero = 0.0;
    const int zi = 0;
    ok = hipMemcpy(da, a, nn * sizeof(double2), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(dn, &n, sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(dextra, &zero, sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(dstat, &zi, sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(djob, &J, sizeof(HeevJob), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(dv, 0, nn * sizeof(double2)) == hipSuccess;
    if (ok) {
      launch_heev(nullptr, djob, 1, n);
      ok = hipDeviceSynchronize() == hipSuccess && hipGetLastError() == hipSuccess &&
           hipMemcpy(w, dw, n * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(v, dv, nn * sizeof(double2), hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(nvec, dnvec, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess;
      if (ok && tri) ok = hipMemcpy(tri, dtri, 2 * n * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
      if (ok && z) ok = hipMemcpy(z, dz, nn * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
    }
  }
  if (!ok) st = PT_TEBD_EDEVICE;
  hipFree(da); hipFree(drefl); hipFree(dv); hipFree(dw); hipFree(dtri); hipFree(dwork); hipFree(dz);
  hipFree(dextra); hipFree(dn); hipFree(dnvec); hipFree(dstat); hipFree(djob);
  return st;
}
}  // namespace

extern "C" pt_tebd_status pt_test_heev(int32_t n, const double* a, int32_t rule, double eps, int32_t cap,
                                       double* w, double* v, int32_t* nvec) {
  return test_heev(n, a, rule, eps, cap, w, v, nvec, nullptr, nullptr);
}

extern "C" pt_tebd_status pt_test_heev_profile(int32_t n, const double* a, int32_t rule, double eps, int32_t reps,
                                               double* stage_ms) {
  if (n < 1 || n > 1024 || !a || !stage_ms || reps < 1) return PT_TEBD_EINVAL;
  const size_t nn = (size_t)n * n;
  double2 *da = nullptr, *da0 = nullptr, *drefl = nullptr, *dv = nullptr;
  double *dw = nullptr, *dtri = nullptr, *dwork = nullptr, *dz = nullptr, *dextra = nullptr;
  int *dn = nullptr, *dnvec = nullptr, *dstat = nullptr;
  unsigned long long* dst = nullptr;
  HeevJob* djob = nullptr;
  bool ok = hipMalloc(&da, nn * sizeof(double2)) == hipSuccess && hipMalloc(&da0, nn * sizeof(double2)) == hipSuccess &&
            hipMalloc(&drefl, nn * sizeof(double2)) == hipSuccess && hipMalloc(&dv, nn * sizeof(double2)) == hipSuccess &&
            hipMalloc(&dw, n * sizeof(double)) == hipSuccess && hipMalloc(&dtri, 6 * n * sizeof(double)) == hipSuccess &&
            hipMalloc(&dwork, 8 * nn * sizeof(double)) == hipSuccess && hipMalloc(&dz, nn * sizeof(double)) == hipSuccess &&
            hipMalloc(&dextra, sizeof(double)) == hipSuccess && hipMalloc(&dn, sizeof(int)) == hipSuccess &&
            hipMalloc(&dnvec, sizeof(int)) == hipSuccess && hipMalloc(&dstat, sizeof(int)) == hipSuccess &&
            hipMalloc(&dst, 8 * sizeof(unsigned long long)) == hipSuccess && hipMalloc(&djob, sizeof(HeevJob)) == hipSuccess;
  int rate_khz = 0;
  ok = ok && hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, 0) == hipSuccess && rate_khz > 0;
  for (int i = 0; i < 9; ++i) stage_ms[i] = 0.0;
  if (ok) {
    HeevJob J{};
    const int r = rule == 0 ? ptt::RULE_ALL : rule == 1 ? ptt::RULE_EPS : rule == 2 ? ptt::RULE_CAP
                : rule == 3 ? ptt::RULE_RANK : ptt::RULE_FULL;
    fill_heev(J, da, n, dn, dw, drefl, dtri, dwork, dz, n, dnvec, r, eps, 0, dextra, eps, dv, n, ptt::SCALE_NONE, dstat);
    J.stamps = dst;
    const double zero = 0.0;
    const int zi = 0;
    ok = hipMemcpy(da0, a, nn * sizeof(double2), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(dn, &n, sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(dextra, &zero, sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(dstat, &zi, sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(djob, &J, sizeof(HeevJob), hipMemcpyHostToDevice) == hipSuccess;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess && hipEventCreate(&e2) == hipSuccess;
    for (int rep = 0; rep < reps && ok; ++rep) {
      ok = hipMemcpy(da, da0, nn * sizeof(double2), hipMemcpyDeviceToDevice) == hipSuccess;
      hipEventRecord(e0, nullptr);
      ptt::heev_tridiag_kernel<<<1, ptt::HEEV_TRI_THREADS, 0, nullptr>>>(djob, nullptr);
      ptt::heev_solve_kernel<<<1, ptt::HEEV_SOLVE_THREADS, 0, nullptr>>>(djob);
      hipEventRecord(e1, nullptr);
      // back-transformation and the two orthonormalisation passes
      dim3 grid((n + ptt::HEEV_BT_COLS - 1) / ptt::HEEV_BT_COLS, 1);
      ptt::heev_backtransform_kernel<<<grid, ptt::HEEV_THREADS, (size_t)n * ptt::HEEV_BT_COLS * sizeof(double2), nullptr>>>(djob);
      const int tiles = (n + ptt::GEMM_BM - 1) / ptt::GEMM_BM;
      for (int pass = 0; pass < 2; ++pass) {
        ptt::heev_orth_gemm<<<dim3(tiles, tiles, 1), ptt::GEMM_THREADS, 0, nullptr>>>(djob, 0);
        ptt::heev_orth_mfix<<<dim3(elem_blocks((long long)n * n), 1), kThreads, 0, nullptr>>>(djob);
        ptt::heev_orth_gemm<<<dim3(tiles, tiles, 1), ptt::GEMM_THREADS, 0, nullptr>>>(djob, 1);
        ptt::heev_orth_norm<<<dim3((n + 63) / 64, 1), 256, 0, nullptr>>>(djob, 1, pass == 1);
      }
      hipEventRecord(e2, nullptr);
      unsigned long long t[8];
      float ms_solve = 0.f, ms_rest = 0.f;
      ok = ok && hipDeviceSynchronize() == hipSuccess &&
           hipMemcpy(t, dst, 7 * sizeof(unsigned long long), hipMemcpyDeviceToHost) == hipSuccess &&
           hipEventElapsedTime(&ms_solve, e0, e1) == hipSuccess && hipEventElapsedTime(&ms_rest, e1, e2) == hipSuccess;
      if (!ok) break;
      for (int i = 0; i < 6; ++i) stage_ms[i] += (double)(t[i + 1] - t[i]) / rate_khz / reps;
      stage_ms[6] += ms_solve / reps;
      stage_ms[7] += ms_rest / reps;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e2) hipEventDestroy(e2);
  }
  hipFree(da); hipFree(da0); hipFree(drefl); hipFree(dv); hipFree(dw); hipFree(dtri); hipFree(dwork); hipFree(dz);
  hipFree(dextra); hipFree(dn); hipFree(dnvec); hipFree(dstat); hipFree(dst); hipFree(djob);
  return ok ? PT_TEBD_OK : PT_TEBD_EDEVICE;
}

extern "C" pt_tebd_status pt_test_heev_tridiagonal(int32_t n, const double* a, int32_t rule, double eps, int32_t cap,
                                                   double* w, double* v, int32_t* nvec, double* tri, double* z) {
  if (!tri || !z) return PT_TEBD_EINVAL;
  return test_heev(n, a, rule, eps, cap, w, v, nvec, tri, z);
}

// ------------------------------------------------------- no-alloc variant
// pt_heev_noalloc: the eigensolver of pt_test_heev on caller-owned device
// buffers, with every other buffer carved out of one file-scope device
// array.  Host code never passes the array's name to a kernel: the device
// address of each GPU's copy is taken once per device with
// hipGetSymbolAddress and kept.
namespace {
constexpr int NOALLOC_NMAX = 256;
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t NOALLOC_BYTES =
    align256(sizeof(HeevJob)) + align256(4 * sizeof(int)) + align256(sizeof(double)) +
    2 * align256((size_t)NOALLOC_NMAX * NOALLOC_NMAX * sizeof(double2)) +  // matrix copy, reflectors
    align256(6 * (size_t)NOALLOC_NMAX * sizeof(double)) +                  // tridiagonal
    align256(8 * (size_t)NOALLOC_NMAX * NOALLOC_NMAX * sizeof(double)) +   // inverse-iteration work
    align256((size_t)NOALLOC_NMAX * NOALLOC_NMAX * sizeof(double));         // tridiagonal eigenvectors
}  // namespace

static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of this device's scratch (set up once per device)
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// scratch layout and the zeroed / copied inputs of one call
__global__ void k_noalloc_setup(char* base, int n, const double2* a_in, int rule, double eps, int cap, double* w,
                                double2* v) {
  size_t off = 0;
  auto take = [&](size_t b) { char* p = base + off; off += align256(b); return p; };
  HeevJob* job = reinterpret_cast<HeevJob*>(take(sizeof(HeevJob)));
  int* ints = reinterpret_cast<int*>(take(4 * sizeof(int)));            // n, nvec, status, pad
  double* extra = reinterpret_cast<double*>(take(sizeof(double)));
  double2* a = reinterpret_cast<double2*>(take((size_t)NOALLOC_NMAX * NOALLOC_NMAX * sizeof(double2)));
  double2* refl = reinterpret_cast<double2*>(take((size_t)NOALLOC_NMAX * NOALLOC_NMAX * sizeof(double2)));
  double* tri = reinterpret_cast<double*>(take(6 * (size_t)NOALLOC_NMAX * sizeof(double)));
  double* work = reinterpret_cast<double*>(take(8 * (size_t)NOALLOC_NMAX * NOALLOC_NMAX * sizeof(double)));
  double* z = reinterpret_cast<double*>(take((size_t)NOALLOC_NMAX * NOALLOC_NMAX * sizeof(double)));
  const long long tot = (long long)n * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x)
    a[i] = a_in[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ints[0] = n;
    ints[1] = 0;
    ints[2] = 0;
    *extra = 0.0;
    HeevJob J{};
    J.a = a; J.lda = n; J.n_ptr = ints; J.refl = refl; J.tri = tri; J.work = work; J.z = z;
    J.n_cap = n; J.nvec_out = ints + 1; J.rule = rule; J.eps = eps; J.cap = cap; J.extra_tail = extra;
    J.rank_tol = eps; J.v = v; J.ldv = n; J.scale = ptt::SCALE_NONE; J.status = ints + 2;
    J.noise_cluster = 1; J.abs_ref = nullptr; J.abs_tol = 0.0; J.w = w;
    *job = J;
  }
}

// number of selected vectors and the eigensolver's status word, to the caller
__global__ void k_noalloc_finish(const char* base, int* nvec_out, int* status_out) {
  const int* ints = reinterpret_cast<const int*>(base + align256(sizeof(HeevJob)));
  *nvec_out = ints[1];
  *status_out = ints[2];
}
}  // namespace

extern "C" pt_tebd_status pt_heev_noalloc(int32_t n, const double* a_dev, int32_t rule, double eps, int32_t cap,
                                          double* w_dev, double* v_dev, int32_t* nvec_dev, int32_t* status_dev,
                                          void* hip_stream) {
  if (n < 1 || n > NOALLOC_NMAX || !a_dev || !w_dev || !v_dev || !nvec_dev || !status_dev) return PT_TEBD_EINVAL;
  if (rule < 0 || rule > 4) return PT_TEBD_EINVAL;
  void* base = nullptr;
  if (scratch_address(&base) != hipSuccess) return PT_TEBD_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int r = rule == 0 ? ptt::RULE_ALL : rule == 1 ? ptt::RULE_EPS : rule == 2 ? ptt::RULE_CAP
              : rule == 3 ? ptt::RULE_RANK : ptt::RULE_FULL;
  char* b = static_cast<char*>(base);
  k_noalloc_setup<<<elem_blocks((long long)n * n), kThreads, 0, st>>>(
      b, n, reinterpret_cast<const double2*>(a_dev), r, eps, cap, w_dev, reinterpret_cast<double2*>(v_dev));
  launch_heev(st, reinterpret_cast<const HeevJob*>(b), 1, n);
  k_noalloc_finish<<<1, 1, 0, st>>>(b, nvec_dev, status_dev);
  return hipGetLastError() == hipSuccess ? PT_TEBD_OK : PT_TEBD_EDEVICE;
}
