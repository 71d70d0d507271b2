// Host-side double-precision helpers of the PT-TEBD library (see host_math.h).
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace ptt {

namespace {

inline cplx cj(cplx z) { return std::conj(z); }

double norm1(int n, const cplx* a) {
  double best = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::abs(a[i * n + j]);
    best = std::max(best, s);
  }
  return best;
}

}  // namespace

std::vector<cplx> matmul(int n, int k, int m, const cplx* a, const cplx* b) {
  std::vector<cplx> c(static_cast<size_t>(n) * m, cplx(0.0));
  for (int i = 0; i < n; ++i)
    for (int p = 0; p < k; ++p) {
      const cplx aip = a[i * k + p];
      if (aip == cplx(0.0)) continue;
      for (int j = 0; j < m; ++j) c[i * m + j] += aip * b[p * m + j];
    }
  return c;
}

std::vector<cplx> expm(int n, const cplx* a) {
  // scale so that the Taylor series converges fast, then square back
  const double nrm = norm1(n, a);
  int squarings = 0;
  double scale = 1.0;
  while (nrm * scale > 0.25) {
    scale *= 0.5;
    ++squarings;
  }
  std::vector<cplx> x(a, a + static_cast<size_t>(n) * n);
  for (auto& v : x) v *= scale;
  std::vector<cplx> sum(static_cast<size_t>(n) * n, cplx(0.0)), term(sum);
  for (int i = 0; i < n; ++i) sum[i * n + i] = term[i * n + i] = 1.0;
  for (int k = 1; k < 40; ++k) {
    term = matmul(n, n, n, term.data(), x.data());
    const double inv = 1.0 / k;
    double tn = 0.0;
    for (size_t i = 0; i < term.size(); ++i) {
      term[i] *= inv;
      sum[i] += term[i];
      tn = std::max(tn, std::abs(term[i]));
    }
    if (tn < 1e-20) break;
  }
  for (int s = 0; s < squarings; ++s) sum = matmul(n, n, n, sum.data(), sum.data());
  return sum;
}

// ---------------------------------------------------------------------------
// Hermitian eigensolver.
//
// Reduction: for column j, a reflector H_j = I - tau v v^H (v_0 = 1) with
// H_j^H x = beta e_1, beta real, acting on rows/cols j+1..n-1, so that
// Q^H A Q = T is real tridiagonal with Q = H_0 H_1 ... H_{n-2}.
// Tridiagonal stage: implicit-shift QL sweeps (Wilkinson shift) with Givens
// rotations accumulated into Z, the tql2 scheme of Bowdler, Martin, Reinsch
// and Wilkinson (Numer. Math. 11, 1968) written out here; eigenvectors of A
// are Q Z.
bool heev(int n, const cplx* ain, double* w, cplx* v) {
  std::vector<cplx> a(ain, ain + static_cast<size_t>(n) * n);
  std::vector<double> d(n, 0.0), e(std::max(n, 1), 0.0);
  std::vector<cplx> taus(std::max(n - 1, 1), cplx(0.0));
  std::vector<cplx> y(n), wv(n);
  for (int j = 0; j + 1 < n; ++j) {
    const int m = n - j - 1;
    cplx alpha = a[(j + 1) * n + j];
    double sig2 = 0.0;
    for (int i = 1; i < m; ++i) sig2 += std::norm(a[(j + 1 + i) * n + j]);
    cplx tau(0.0);
    double beta = alpha.real();
    if (!(sig2 == 0.0 && alpha.imag() == 0.0)) {
      const double nrm = std::sqrt(std::norm(alpha) + sig2);
      beta = alpha.real() >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      const cplx scal = 1.0 / (alpha - beta);
      for (int i = 1; i < m; ++i) a[(j + 1 + i) * n + j] *= scal;
    }
    taus[j] = tau;
    e[j] = beta;
    a[(j + 1) * n + j] = 1.0;  // v_0 (restored below)
    if (tau != cplx(0.0)) {
      // y = tau * A22 v ;  w = y - 1/2 (conj(tau) v^H y) v ;  A22 -= w v^H + v w^H
      for (int r = 0; r < m; ++r) {
        cplx s(0.0);
        for (int c = 0; c < m; ++c) s += a[(j + 1 + r) * n + (j + 1 + c)] * a[(j + 1 + c) * n + j];
        y[r] = tau * s;
      }
      cplx vhy(0.0);
      for (int r = 0; r < m; ++r) vhy += cj(a[(j + 1 + r) * n + j]) * y[r];
      const double half = 0.5 * (cj(tau) * vhy).real();
      for (int r = 0; r < m; ++r) wv[r] = y[r] - half * a[(j + 1 + r) * n + j];
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
          const cplx vr = a[(j + 1 + r) * n + j], vc = a[(j + 1 + c) * n + j];
          a[(j + 1 + r) * n + (j + 1 + c)] -= wv[r] * cj(vc) + vr * cj(wv[c]);
        }
    }
  }
  for (int j = 0; j < n; ++j) d[j] = a[j * n + j].real();
  if (n > 0) e[n - 1] = 0.0;

  // Q = H_0 ... H_{n-2}: apply to the identity from the innermost reflector
  std::vector<cplx> q(static_cast<size_t>(n) * n, cplx(0.0));
  for (int i = 0; i < n; ++i) q[i * n + i] = 1.0;
  for (int j = n - 2; j >= 0; --j) {
    const cplx tau = taus[j];
    if (tau == cplx(0.0)) continue;
    const int m = n - j - 1;
    auto vv = [&](int i) { return i == 0 ? cplx(1.0) : a[(j + 1 + i) * n + j]; };
    for (int c = 0; c < n; ++c) {
      cplx s(0.0);
      for (int i = 0; i < m; ++i) s += cj(vv(i)) * q[(j + 1 + i) * n + c];
      s *= tau;
      for (int i = 0; i < m; ++i) q[(j + 1 + i) * n + c] -= s * vv(i);
    }
  }

  // implicit QL on (d, e); e[i] couples i and i+1
  std::vector<double> z(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) z[i * n + i] = 1.0;
  for (int lo = 0; lo < n; ++lo) {
    int sweeps = 0;
    while (true) {
      int m = lo;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 2.2e-16 * dd) break;
      }
      if (m == lo) break;
      if (++sweeps > 80) return false;
      double g = (d[lo + 1] - d[lo]) / (2.0 * e[lo]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[lo] + e[lo] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool early = false;
      for (int i = m - 1; i >= lo; --i) {
        double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          const double zf = z[k * n + i + 1];
          z[k * n + i + 1] = s * z[k * n + i] + c * zf;
          z[k * n + i] = c * z[k * n + i] - s * zf;
        }
      }
      if (early) continue;
      d[lo] -= p;
      e[lo] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y2) { return d[x] < d[y2]; });
  for (int kk = 0; kk < n; ++kk) {
    const int src = order[kk];
    w[kk] = d[src];
    for (int i = 0; i < n; ++i) {
      cplx s(0.0);
      for (int p = 0; p < n; ++p) s += q[i * n + p] * z[p * n + src];
      v[i * n + kk] = s;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Chain propagators.

namespace {

// -i (H kron 1 - 1 kron H^T) on an m-dimensional Hilbert space
void add_hamiltonian_part(int m, const cplx* h, cplx* lsup) {
  const int mm = m * m;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) {
          cplx val(0.0);
          if (j == l) val += h[i * m + k];
          if (i == k) val -= h[l * m + j];  // (H^T)[j][l] = H[l][j]
          lsup[(i * m + j) * mm + (k * m + l)] += cplx(0.0, -1.0) * val;
        }
}

// w * [L kron conj(L) - 1/2 (L^dag L kron 1 + 1 kron (L^dag L)^T)]
void add_gksl_part(int m, const cplx* lop, double wgt, cplx* lsup) {
  const int mm = m * m;
  std::vector<cplx> ldl(static_cast<size_t>(m) * m, cplx(0.0));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int p = 0; p < m; ++p) ldl[i * m + j] += std::conj(lop[p * m + i]) * lop[p * m + j];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) {
          cplx val = lop[i * m + k] * std::conj(lop[j * m + l]);
          if (j == l) val -= 0.5 * ldl[i * m + k];
          if (i == k) val -= 0.5 * ldl[l * m + j];
          lsup[(i * m + j) * mm + (k * m + l)] += wgt * val;
        }
}

void kron(int m1, const cplx* a, int m2, const cplx* b, cplx* out) {
  const int m = m1 * m2;
  for (int i1 = 0; i1 < m1; ++i1)
    for (int j1 = 0; j1 < m1; ++j1)
      for (int i2 = 0; i2 < m2; ++i2)
        for (int j2 = 0; j2 < m2; ++j2)
          out[(i1 * m2 + i2) * m + (j1 * m2 + j2)] = a[i1 * m1 + j1] * b[i2 * m2 + j2];
}

}  // namespace

std::vector<std::vector<cplx>> chain_gates(int n_sites, int d, double dt, const cplx* h_site,
                                           const cplx* h_bond, int n_lind, const cplx* lindblad) {
  std::vector<std::vector<cplx>> out;
  const int d2 = d * d;
  std::vector<cplx> eye(static_cast<size_t>(d) * d, cplx(0.0));
  for (int i = 0; i < d; ++i) eye[i * d + i] = 1.0;
  if (n_sites == 1) {
    std::vector<cplx> lsup(static_cast<size_t>(d2) * d2, cplx(0.0));
    add_hamiltonian_part(d, h_site, lsup.data());
    for (int k = 0; k < n_lind; ++k) add_gksl_part(d, lindblad + static_cast<size_t>(k) * d * d, 1.0, lsup.data());
    for (auto& x : lsup) x *= 0.5 * dt;
    out.push_back(expm(d2, lsup.data()));
    return out;
  }
  const int m = d2, mm = m * m;  // two-site Hilbert dim d^2, Liouville dim d^4
  for (int b = 0; b + 1 < n_sites; ++b) {
    // weights with which the two site terms enter K' (first and last bonds
    // carry the whole end-site term; N = 2 carries both whole terms)
    double wl = 0.5, wr = 0.5;
    if (n_sites == 2) {
      wl = wr = 1.0;
    } else {
      if (b == 0) wl = 1.0;
      if (b == n_sites - 2) wr = 1.0;
    }
    std::vector<cplx> kp(h_bond + static_cast<size_t>(b) * m * m, h_bond + static_cast<size_t>(b + 1) * m * m);
    std::vector<cplx> tmp(static_cast<size_t>(m) * m);
    kron(d, h_site + static_cast<size_t>(b) * d * d, d, eye.data(), tmp.data());
    for (int i = 0; i < m * m; ++i) kp[i] += wl * tmp[i];
    kron(d, eye.data(), d, h_site + static_cast<size_t>(b + 1) * d * d, tmp.data());
    for (int i = 0; i < m * m; ++i) kp[i] += wr * tmp[i];
    std::vector<cplx> lnat(static_cast<size_t>(mm) * mm, cplx(0.0));
    add_hamiltonian_part(m, kp.data(), lnat.data());
    for (int side = 0; side < 2; ++side) {
      const int site = b + side;
      const double wgt = side == 0 ? wl : wr;
      for (int k = 0; k < n_lind; ++k) {
        const cplx* lop = lindblad + (static_cast<size_t>(site) * n_lind + k) * d * d;
        if (side == 0) kron(d, lop, d, eye.data(), tmp.data());
        else kron(d, eye.data(), d, lop, tmp.data());
        add_gksl_part(m, tmp.data(), wgt, lnat.data());
      }
    }
    // natural (i1 i2),(j1 j2) -> site-major (i1 j1),(i2 j2)
    std::vector<int> perm(mm);
    for (int i1 = 0; i1 < d; ++i1)
      for (int j1 = 0; j1 < d; ++j1)
        for (int i2 = 0; i2 < d; ++i2)
          for (int j2 = 0; j2 < d; ++j2)
            perm[((i1 * d + j1) * d + i2) * d + j2] = ((i1 * d + i2) * d + j1) * d + j2;
    const double tau = (b % 2 == 0) ? 0.5 * dt : 0.25 * dt;
    std::vector<cplx> lsm(static_cast<size_t>(mm) * mm);
    for (int r = 0; r < mm; ++r)
      for (int c = 0; c < mm; ++c) lsm[r * mm + c] = lnat[perm[r] * mm + perm[c]] * tau;
    out.push_back(expm(mm, lsm.data()));
  }
  return out;
}

// ---------------------------------------------------------------------------
// Bath influence coefficients.

namespace {

// ln|Gamma(z)| for Re z > 0: shift up to Re z >= 12, then the Stirling series.
double log_abs_gamma(cplx z) {
  double shift = 0.0;
  while (z.real() < 12.0) {
    shift += std::log(std::abs(z));
    z += 1.0;
  }
  // (z - 1/2) ln z - z + 1/2 ln(2 pi) + sum_k B_2k / (2k (2k-1) z^(2k-1))
  static const double bern[] = {1.0 / 6.0, -1.0 / 30.0, 1.0 / 42.0, -1.0 / 30.0,
                                5.0 / 66.0, -691.0 / 2730.0, 7.0 / 6.0};
  cplx s = (z - 0.5) * std::log(z) - z + 0.5 * std::log(2.0 * M_PI);
  cplx zpow = z;
  const cplx z2 = z * z;
  for (int k = 1; k <= 7; ++k) {
    s += bern[k - 1] / (2.0 * k * (2.0 * k - 1.0) * zpow);
    zpow *= z2;
  }
  return s.real() - shift;
}

// G(t) for J = 2 alpha w exp(-w/wc): closed form
cplx g_exp_cutoff(double t, double alpha, double wc, double temperature) {
  const double im = 2.0 * alpha * (std::atan(wc * t) - wc * t);
  double re = alpha * std::log1p(wc * t * wc * t);
  if (temperature > 0.0) {
    const double x = temperature / wc, y = temperature * t;
    re += 4.0 * alpha * (log_abs_gamma(cplx(1.0 + x, 0.0)) - log_abs_gamma(cplx(1.0 + x, y)));
  }
  return {re, im};
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

bool bath_eta(double alpha, double wc, int cutoff_kind, double temperature, double dt, int k_cut,
              std::vector<cplx>& eta, std::string& err) {
  if (!(alpha >= 0.0) || !(wc > 0.0) || !(temperature >= 0.0) || !(dt > 0.0) || k_cut < 0) {
    err = "invalid bath parameters";
    return false;
  }
  eta.assign(k_cut + 1, cplx(0.0));
  if (cutoff_kind == 0) {
    std::vector<cplx> g(k_cut + 2);
    for (int j = 0; j <= k_cut + 1; ++j) g[j] = g_exp_cutoff(j * dt, alpha, wc, temperature);
    eta[0] = g[1];
    for (int k = 1; k <= k_cut; ++k) eta[k] = g[k + 1] - 2.0 * g[k] + g[k - 1];
    return true;
  }
  if (cutoff_kind != 1) {
    err = "cutoff_kind must be 0 (exponential) or 1 (Gaussian)";
    return false;
  }
  // Gaussian cutoff: composite Gauss-Legendre over (0, 7.5 wc)
  std::vector<double> gx, gw;
  gauss_legendre(24, gx, gw);
  const double wmax = 7.5 * wc;
  const double tmax = (k_cut + 1) * dt;
  const int pieces = static_cast<int>(std::ceil(wmax * std::max(tmax, 1.0) / M_PI)) * 2 + 8;
  auto jw = [&](double w) { return 2.0 * alpha * w * std::exp(-(w / wc) * (w / wc)); };
  auto cth = [&](double w) { return temperature > 0.0 ? 1.0 / std::tanh(w / (2.0 * temperature)) : 1.0; };
  for (int p = 0; p < pieces; ++p) {
    const double lo = wmax * p / pieces, hi = wmax * (p + 1) / pieces;
    for (int q = 0; q < 24; ++q) {
      const double w = 0.5 * (hi - lo) * gx[q] + 0.5 * (hi + lo);
      const double wt = 0.5 * (hi - lo) * gw[q];
      const double jw2 = jw(w) / (w * w), c = cth(w);
      // eta_0 = G(dt)
      const double sh = std::sin(0.5 * w * dt);
      eta[0] += wt * jw2 * cplx(c * 2.0 * sh * sh, std::sin(w * dt) - w * dt);
      const double pref = wt * jw2 * 4.0 * sh * sh;
      for (int k = 1; k <= k_cut; ++k)
        eta[k] += pref * cplx(c * std::cos(w * k * dt), -std::sin(w * k * dt));
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// PT-MPO construction: the influence functional is kept as an MPS over time
// slots; slot k enters with its same-step factor, then the factors coupling
// it to the K previous slots are multiplied in (a bond-d^2 copy chain that
// carries x_k back through the window) and the window is recompressed
// (right-to-left orthonormalisation, left-to-right truncated SVD).

namespace {

struct Slot {
  int a = 1, c = 1;        // left/right bond
  std::vector<cplx> t;     // [a][x][c]
};

// Householder QR of a (rows x cols, row-major): a = Q R, Q rows x k with
// orthonormal columns, R k x cols upper triangular, k = min(rows, cols).
// Reflector H_j = I - tau_j v_j v_j^H with H_j^H x = beta e_1.
void householder_qr(int rows, int cols, const std::vector<cplx>& a, std::vector<cplx>& q,
                    std::vector<cplx>& r) {
  std::vector<cplx> m(a);
  const int k = std::min(rows, cols);
  std::vector<std::vector<cplx>> vs(k);
  std::vector<cplx> taus(k, cplx(0.0));
  for (int j = 0; j < k; ++j) {
    const cplx alpha = m[static_cast<size_t>(j) * cols + j];
    double sig = 0.0;
    for (int i = j + 1; i < rows; ++i) sig += std::norm(m[static_cast<size_t>(i) * cols + j]);
    if (sig == 0.0 && alpha.imag() == 0.0) continue;  // column already reduced
    const double nrm = std::sqrt(std::norm(alpha) + sig);
    const double beta = alpha.real() >= 0.0 ? -nrm : nrm;
    const cplx tau = (beta - alpha) / beta;
    const cplx scal = 1.0 / (alpha - beta);
    std::vector<cplx> v(rows - j);
    v[0] = 1.0;
    for (int i = 1; i < rows - j; ++i) v[i] = m[static_cast<size_t>(j + i) * cols + j] * scal;
    for (int c = j; c < cols; ++c) {  // m[j:, c] <- H^H m[j:, c]
      cplx acc(0.0);
      for (int i = 0; i < rows - j; ++i) acc += std::conj(v[i]) * m[static_cast<size_t>(j + i) * cols + c];
      acc *= std::conj(tau);
      for (int i = 0; i < rows - j; ++i) m[static_cast<size_t>(j + i) * cols + c] -= v[i] * acc;
    }
    vs[j] = std::move(v);
    taus[j] = tau;
  }
  r.assign(static_cast<size_t>(k) * cols, cplx(0.0));
  for (int i = 0; i < k; ++i)
    for (int c = i; c < cols; ++c) r[static_cast<size_t>(i) * cols + c] = m[static_cast<size_t>(i) * cols + c];
  q.assign(static_cast<size_t>(rows) * k, cplx(0.0));
  for (int i = 0; i < k; ++i) q[static_cast<size_t>(i) * k + i] = 1.0;
  for (int j = k - 1; j >= 0; --j) {  // Q = H_0 H_1 ... H_{k-1} I
    if (taus[j] == cplx(0.0)) continue;
    const auto& v = vs[j];
    for (int c = 0; c < k; ++c) {
      cplx acc(0.0);
      for (int i = 0; i < rows - j; ++i) acc += std::conj(v[i]) * q[static_cast<size_t>(j + i) * k + c];
      acc *= taus[j];
      for (int i = 0; i < rows - j; ++i) q[static_cast<size_t>(j + i) * k + c] -= v[i] * acc;
    }
  }
}

// One-sided Jacobi from the left on the rows of a (n x m): a = U W with U
// unitary (n x n, accumulated from the plane rotations) and the rows of W
// (returned in a) mutually orthogonal.  U is exactly unitary up to rounding
// however small the row norms are, and W is never divided by anything.
void row_jacobi(int n, int m, std::vector<cplx>& a, std::vector<cplx>& u) {
  u.assign(static_cast<size_t>(n) * n, cplx(0.0));
  for (int i = 0; i < n; ++i) u[static_cast<size_t>(i) * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p + 1 < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        cplx* ap = &a[static_cast<size_t>(p) * m];
        cplx* aq = &a[static_cast<size_t>(q) * m];
        double al = 0.0, be = 0.0;
        cplx c(0.0);
        for (int j = 0; j < m; ++j) {
          al += std::norm(ap[j]);
          be += std::norm(aq[j]);
          c += ap[j] * std::conj(aq[j]);
        }
        const double ac = std::abs(c);
        if (ac == 0.0 || ac <= 1e-16 * std::sqrt(al * be)) continue;
        off = std::max(off, ac / std::sqrt(al * be));
        // rows (p, q) <- G (p, q), G = [[cs, -sn ph], [sn conj(ph), cs]],
        // with tan(theta) = t the smaller root of t^2 + 2 zeta t - 1 = 0
        const cplx ph = c / ac;
        const double zeta = (be - al) / (2.0 * ac);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::hypot(1.0, zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int j = 0; j < m; ++j) {
          const cplx x = ap[j], y = aq[j];
          ap[j] = cs * x - sn * ph * y;
          aq[j] = sn * std::conj(ph) * x + cs * y;
        }
        for (int i = 0; i < n; ++i) {  // U <- U G^H
          cplx& up = u[static_cast<size_t>(i) * n + p];
          cplx& uq = u[static_cast<size_t>(i) * n + q];
          const cplx x = up, y = uq;
          up = cs * x - sn * std::conj(ph) * y;
          uq = sn * ph * x + cs * y;
        }
      }
    if (off < 1e-15) break;
  }
}

// Truncated SVD of a (rows x cols) matrix: QR of the matrix (or of its
// conjugate transpose), then one-sided Jacobi on the small triangular
// factor.  Singular values are the norms of the orthogonalised rows, the
// left factor is a product of unitary factors, and S V^H is formed without
// dividing by any singular value.  Truncation: the smallest rank whose
// discarded tail has 2-norm below eps * sigma_max, then the cap.
// Returns keep and fills u (rows x keep) and svh = S V^H (keep x cols).
int truncated_svd(int rows, int cols, const std::vector<cplx>& m, double eps, int cap,
                  std::vector<cplx>& u, std::vector<cplx>& svh) {
  const int n = std::min(rows, cols);
  std::vector<cplx> ufull, w, qf, rf, u1;
  if (rows >= cols) {  // m = Q R, R = U1 W  ->  m = (Q U1) W
    householder_qr(rows, cols, m, qf, rf);
    row_jacobi(n, cols, rf, u1);
    ufull = matmul(rows, n, n, qf.data(), u1.data());
    w = rf;
  } else {             // m^H = Q R  ->  m = R^H Q^H = U1 W Q^H
    std::vector<cplx> mh(static_cast<size_t>(cols) * rows);
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c) mh[static_cast<size_t>(c) * rows + r] = std::conj(m[static_cast<size_t>(r) * cols + c]);
    householder_qr(cols, rows, mh, qf, rf);  // qf cols x n, rf n x rows
    std::vector<cplx> a(static_cast<size_t>(n) * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) a[static_cast<size_t>(i) * n + j] = std::conj(rf[static_cast<size_t>(j) * rows + i]);
    row_jacobi(n, n, a, u1);
    ufull = u1;
    w.assign(static_cast<size_t>(n) * cols, cplx(0.0));  // W Q^H
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < cols; ++c) {
        cplx acc(0.0);
        for (int k = 0; k < n; ++k) acc += a[static_cast<size_t>(i) * n + k] * std::conj(qf[static_cast<size_t>(c) * n + k]);
        w[static_cast<size_t>(i) * cols + c] = acc;
      }
  }
  std::vector<double> sv(n);
  for (int i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int c = 0; c < cols; ++c) acc += std::norm(w[static_cast<size_t>(i) * cols + c]);
    sv[i] = std::sqrt(acc);
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return sv[x] > sv[y]; });
  std::vector<double> s(n);
  for (int i = 0; i < n; ++i) s[i] = sv[order[i]];
  int npos = 0;
  while (npos < n && s[npos] > 0.0) ++npos;
  int keep = std::max(npos, 1);
  if (npos > 0) {
    std::vector<double> tail(npos + 1, 0.0);
    for (int i = npos - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
    for (int c = 1; c < npos; ++c)
      if (std::sqrt(tail[c]) < eps * s[0]) {
        keep = c;
        break;
      }
  }
  if (cap > 0) keep = std::min(keep, cap);
  keep = std::min(keep, n);
  u.assign(static_cast<size_t>(rows) * keep, cplx(0.0));
  svh.assign(static_cast<size_t>(keep) * cols, cplx(0.0));
  for (int k = 0; k < keep; ++k) {
    const int src = order[k];
    for (int r = 0; r < rows; ++r) u[static_cast<size_t>(r) * keep + k] = ufull[static_cast<size_t>(r) * n + src];
    for (int c = 0; c < cols; ++c) svh[static_cast<size_t>(k) * cols + c] = w[static_cast<size_t>(src) * cols + c];
  }
  return keep;
}

void recompress(std::vector<Slot>& mps, int lo, int hi, int d2, double eps, int cap) {
  // right-to-left: slot j = L Q with Q having orthonormal rows (QR of the
  // slot's conjugate transpose, no truncation)
  for (int j = hi; j > lo; --j) {
    Slot& s = mps[j];
    const int rows = s.a, cols = d2 * s.c;
    std::vector<cplx> mh(static_cast<size_t>(cols) * rows);
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c) mh[static_cast<size_t>(c) * rows + r] = std::conj(s.t[static_cast<size_t>(r) * cols + c]);
    std::vector<cplx> qf, rf;  // M^H = Q R  ->  M = R^H Q^H
    householder_qr(cols, rows, mh, qf, rf);
    const int keep = std::min(rows, cols);
    std::vector<cplx> qn(static_cast<size_t>(keep) * cols), lmat(static_cast<size_t>(rows) * keep);
    for (int k = 0; k < keep; ++k)
      for (int c = 0; c < cols; ++c) qn[static_cast<size_t>(k) * cols + c] = std::conj(qf[static_cast<size_t>(c) * keep + k]);
    for (int r = 0; r < rows; ++r)
      for (int k = 0; k < keep; ++k) lmat[static_cast<size_t>(r) * keep + k] = std::conj(rf[static_cast<size_t>(k) * rows + r]);
    s.t = qn;
    s.a = keep;
    Slot& p = mps[j - 1];
    p.t = matmul(p.a * d2, p.c, keep, p.t.data(), lmat.data());
    p.c = keep;
  }
  for (int j = lo; j < hi; ++j) {
    Slot& s = mps[j];
    std::vector<cplx> u, svh;
    const int keep = truncated_svd(s.a * d2, s.c, s.t, eps, cap, u, svh);
    s.t = u;
    s.c = keep;
    Slot& nx = mps[j + 1];
    nx.t = matmul(keep, nx.a, d2 * nx.c, svh.data(), nx.t.data());
    nx.a = keep;
  }
}

}  // namespace

bool build_ptmpo(const std::vector<cplx>& eta, const std::vector<double>& sigma, int n_steps,
                 double eps, int xi_max, std::vector<std::vector<cplx>>& tensors,
                 std::vector<int>& dims, std::string& err) {
  const int d = static_cast<int>(sigma.size());
  const int d2 = d * d;
  const int k_cut = static_cast<int>(eta.size()) - 1;
  if (n_steps < 1 || d < 1 || k_cut < 0) {
    err = "invalid PT-MPO request";
    return false;
  }
  // b[D][x][x'] = exp(-(s+_x - s-_x)(eta_D s+_x' - conj(eta_D) s-_x'))
  std::vector<std::vector<cplx>> b(k_cut + 1, std::vector<cplx>(static_cast<size_t>(d2) * d2));
  for (int dl = 0; dl <= k_cut; ++dl)
    for (int x = 0; x < d2; ++x)
      for (int xp = 0; xp < d2; ++xp) {
        const double spx = sigma[x / d], smx = sigma[x % d];
        const double spy = sigma[xp / d], smy = sigma[xp % d];
        b[dl][x * d2 + xp] = std::exp(-(spx - smx) * (eta[dl] * spy - std::conj(eta[dl]) * smy));
      }
  std::vector<Slot> mps;
  for (int k = 1; k <= n_steps; ++k) {
    Slot ns;
    ns.t.assign(d2, cplx(0.0));
    for (int x = 0; x < d2; ++x) ns.t[x] = b[0][x * d2 + x];
    mps.push_back(ns);
    const int m = std::min(k_cut, k - 1);
    if (m == 0) continue;
    const int last = static_cast<int>(mps.size()) - 1;
    {  // newest slot emits its index on a new left bond (a, xk)
      Slot& s = mps[last];
      std::vector<cplx> t(static_cast<size_t>(s.a) * d2 * d2 * s.c, cplx(0.0));
      for (int a = 0; a < s.a; ++a)
        for (int x = 0; x < d2; ++x)
          for (int c = 0; c < s.c; ++c) t[((a * d2 + x) * d2 + x) * s.c + c] = s.t[(a * d2 + x) * s.c + c];
      s.t = t;
      s.a *= d2;
    }
    for (int dl = 1; dl <= m; ++dl) {
      Slot& s = mps[last - dl];
      const bool through = dl < m;
      const int na = through ? s.a * d2 : s.a, nc = s.c * d2;
      std::vector<cplx> t(static_cast<size_t>(na) * d2 * nc, cplx(0.0));
      for (int a = 0; a < s.a; ++a)
        for (int x = 0; x < d2; ++x)
          for (int c = 0; c < s.c; ++c) {
            const cplx val = s.t[(a * d2 + x) * s.c + c];
            for (int xk = 0; xk < d2; ++xk) {
              const int aa = through ? a * d2 + xk : a;
              t[(aa * d2 + x) * nc + c * d2 + xk] = val * b[dl][xk * d2 + x];
            }
          }
      s.t = t;
      s.a = na;
      s.c = nc;
    }
    recompress(mps, last - m, last, d2, eps, xi_max);
  }
  tensors.clear();
  dims.assign(n_steps + 1, 1);
  for (int k = 0; k < n_steps; ++k) {
    const Slot& s = mps[k];
    std::vector<cplx> p(static_cast<size_t>(s.a) * s.c * d2);
    for (int a = 0; a < s.a; ++a)
      for (int x = 0; x < d2; ++x)
        for (int c = 0; c < s.c; ++c) p[(a * s.c + c) * d2 + x] = s.t[(a * d2 + x) * s.c + c];
    tensors.push_back(p);
    dims[k] = s.a;
    dims[k + 1] = s.c;
  }
  return true;
}

std::vector<std::vector<cplx>> caps_backward(const std::vector<std::vector<cplx>>& tensors,
                                             const std::vector<int>& dims, int d, bool diagonal) {
  const int m = static_cast<int>(tensors.size());
  const int d2 = d * d;
  std::vector<std::vector<cplx>> caps(m + 1);
  caps[m].assign(dims[m], cplx(1.0));
  for (int k = m; k >= 1; --k) {
    const auto& p = tensors[k - 1];
    const int xi_in = dims[k - 1], xi_out = dims[k];
    caps[k - 1].assign(xi_in, cplx(0.0));
    for (int e = 0; e < xi_in; ++e) {
      cplx acc(0.0);
      for (int f = 0; f < xi_out; ++f) {
        cplx red(0.0);
        for (int i = 0; i < d; ++i) {
          const int s = i * d + i;  // diagonal Liouville index (trace vector)
          if (diagonal) {
            red += p[(static_cast<size_t>(e) * xi_out + f) * d2 + s];
          } else {
            for (int i2 = 0; i2 < d; ++i2)
              red += p[((static_cast<size_t>(e) * xi_out + f) * d2 + s) * d2 + (i2 * d + i2)];
          }
        }
        acc += red * caps[k][f];
      }
      caps[k - 1][e] = acc / static_cast<double>(d);
    }
  }
  return caps;
}

}  // namespace ptt
