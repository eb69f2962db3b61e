// Host float64 precompute: PSWF (App. B), Lambert W, Alg. 3, scaling and window tables.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace pswfe {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Number of eigenvalues of the symmetric tridiagonal matrix (diag d, off-diagonal e) below x
// (Sturm sequence count from the LDL^T pivots).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0) ++cnt;
  for (size_t i = 1; i < d.size(); ++i) {
    if (q == 0.0) q = std::numeric_limits<double>::min();
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// Solves (T - shift I) y = b in place for a symmetric tridiagonal T, Gaussian elimination
// with partial pivoting (row interchanges create one extra superdiagonal).
void tridiag_solve(const std::vector<double>& diag, const std::vector<double>& off, double shift,
                   std::vector<double>* rhs) {
  const int n = static_cast<int>(diag.size());
  std::vector<double> dl(off), du(off), d(n), du2(std::max(n - 2, 0), 0.0);
  std::vector<double>& b = *rhs;
  const double tiny = 1e-300;
  for (int i = 0; i < n; ++i) d[i] = diag[i] - shift;
  for (int i = 0; i < n - 1; ++i) {
    if (std::fabs(d[i]) >= std::fabs(dl[i])) {
      if (d[i] == 0.0) d[i] = tiny;
      const double f = dl[i] / d[i];
      d[i + 1] -= f * du[i];
      b[i + 1] -= f * b[i];
    } else {
      const double f = d[i] / dl[i];
      d[i] = dl[i];
      const double t = d[i + 1];
      d[i + 1] = du[i] - f * t;
      if (i < n - 2) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du2[i];
      }
      du[i] = t;
      const double tb = b[i];
      b[i] = b[i + 1];
      b[i + 1] = tb - f * b[i + 1];
    }
  }
  if (d[n - 1] == 0.0) d[n - 1] = tiny;
  b[n - 1] /= d[n - 1];
  if (n > 1) b[n - 2] = (b[n - 2] - du[n - 2] * b[n - 1]) / d[n - 2];
  for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - du[i] * b[i + 1] - du2[i] * b[i + 2]) / d[i];
}

}  // namespace

Pswf::Pswf(double c_) : c(c_) {
  const int K = std::max(40, static_cast<int>(1.5 * c) + 30);
  std::vector<double> d(K), e(K - 1);
  const double c2 = c * c;
  for (int i = 0; i < K; ++i) {
    const double n = 2.0 * i;
    d[i] = n * (n + 1.0) + c2 * (2.0 * n * (n + 1.0) - 1.0) / ((2.0 * n + 3.0) * (2.0 * n - 1.0));
    if (i < K - 1)
      e[i] = c2 * (n + 1.0) * (n + 2.0) / ((2.0 * n + 3.0) * std::sqrt((2.0 * n + 1.0) * (2.0 * n + 5.0)));
  }
  // Gershgorin interval, then bisection on the Sturm count for the smallest eigenvalue.
  double lo = d[0] - std::fabs(e[0]), hi = d[0] + std::fabs(e[0]);
  for (int i = 1; i < K; ++i) {
    const double r = std::fabs(e[i - 1]) + (i < K - 1 ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(d, e, mid) >= 1) hi = mid; else lo = mid;
  }
  chi0 = 0.5 * (lo + hi);
  // Inverse iteration for the eigenvector (orthonormal Legendre basis).
  std::vector<double> v(K, 1.0);
  for (int it = 0; it < 4; ++it) {
    tridiag_solve(d, e, chi0, &v);
    double nrm = 0.0;
    for (double x : v) nrm += x * x;
    nrm = std::sqrt(nrm);
    for (double& x : v) x /= nrm;
  }
  a.resize(K);
  for (int i = 0; i < K; ++i) a[i] = v[i] * std::sqrt(2.0 * i + 0.5);  // Pbar_n = sqrt(n+1/2) P_n
  psi_0 = psi(0.0);
  if (psi_0 < 0) {
    for (double& x : a) x = -x;
    psi_0 = -psi_0;
  }
  psi_1 = psi(1.0);
  lambda0 = 2.0 * a[0] / psi_0;  // int_{-1}^{1} P_0 = 2, other P_n integrate to 0
}

double Pswf::psi(double x) const {
  // Legendre three-term recurrence, summing the even degrees.
  double p0 = 1.0, p1 = x, s = a[0];
  const int nmax = 2 * static_cast<int>(a.size()) - 2;
  for (int n = 1; n < nmax; ++n) {
    const double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
    p0 = p1;
    p1 = p2;
    if ((n + 1) % 2 == 0) s += a[(n + 1) / 2] * p1;
  }
  return s;
}

double Pswf::dpsi(double x) const {
  // P'_{n+1} = P'_{n-1} + (2n+1) P_n
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0, s = 0.0;
  const int nmax = 2 * static_cast<int>(a.size()) - 2;
  for (int n = 1; n < nmax; ++n) {
    const double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
    const double d2 = d0 + (2.0 * n + 1.0) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
    if ((n + 1) % 2 == 0) s += a[(n + 1) / 2] * d1;
  }
  return s;
}

double Pswf::ipsi(double x) const {
  // int_0^x P_0 = x; int_0^x P_n = (P_{n+1}(x) - P_{n-1}(x)) / (2n + 1) for even n >= 2
  // (both values vanish at 0 for odd indices).
  const int nmax = 2 * static_cast<int>(a.size());
  std::vector<double> P(static_cast<size_t>(nmax) + 1);
  P[0] = 1.0;
  if (nmax >= 1) P[1] = x;
  for (int n = 1; n < nmax; ++n) P[n + 1] = ((2.0 * n + 1.0) * x * P[n] - n * P[n - 1]) / (n + 1.0);
  double s = a[0] * x;
  for (size_t k = 1; k < a.size(); ++k) {
    const int n = 2 * static_cast<int>(k);
    s += a[k] * (P[n + 1] - P[n - 1]) / (2.0 * n + 1.0);
  }
  return s;
}

// Halley iteration on f(w) = w e^w - x.
static double halley_w(double x, double w) {
  for (int it = 0; it < 100; ++it) {
    const double ew = std::exp(w);
    const double f = w * ew - x;
    const double fp = ew * (w + 1.0);
    const double dw = f / (fp - (w + 2.0) * f / (2.0 * w + 2.0));
    w -= dw;
    if (std::fabs(dw) <= 1e-15 * (1.0 + std::fabs(w))) break;
  }
  return w;
}

double lambert_w0(double x) {
  if (x == 0.0) return 0.0;
  double w = x < 1.0 ? std::log1p(x) : std::log(x) - std::log(std::max(std::log(x), 1e-3));
  if (x < -0.25) w = -1.0 + std::sqrt(2.0 * (1.0 + std::exp(1.0) * x));
  return halley_w(x, w);
}

double lambert_wm1(double x) {
  double w;
  if (x > -0.25) {
    const double l1 = std::log(-x);
    w = l1 - std::log(-l1);
  } else {
    w = -1.0 - std::sqrt(std::max(0.0, 2.0 * (1.0 + std::exp(1.0) * x)));
  }
  return halley_w(x, w);
}

bool is_smooth_even(int m) {
  if (m < 2 || (m & 1)) return false;
  for (int p : {2, 3, 5, 7})
    while (m % p == 0) m /= p;
  return m == 1;
}

int next_smooth_even(int m) {
  m = std::max(m, 2);
  while (!is_smooth_even(m)) ++m;
  return m;
}

namespace {
constexpr double kAs = 5.0;  // split-model prefactor (Sec. 5.1.1)
double as_over_aw() { return 4.0 * std::sqrt(5.0) / std::pow(kPi, 1.5); }  // Sec. 6.3

double cs_of(double eps, double L, double rc, double q_l2, int tol_mode) {
  if (tol_mode == 0) return std::log(1.0 / eps);
  const double Bs = kAs * q_l2 * std::sqrt(rc) / std::sqrt(L * L * L);  // eq. cs_dimless
  const double r = Bs / eps;
  return 0.5 * lambert_w0(2.0 * r * r);
}
}  // namespace

int choose_params(double eps, double L, double rc, int m, int64_t n, double q_l2, int tol_mode,
                  Params* out) {
  if (!out || !(L > 0.0) || !std::isfinite(L) || (tol_mode != 0 && tol_mode != 1)) return 1;
  if (!(eps >= 1e-14 && eps <= 0.1)) return 2;
  if (tol_mode == 1 && !(q_l2 > 0.0 && std::isfinite(q_l2))) return 1;
  if (m > 0 && (!is_smooth_even(m) || m < 8 || m > 512)) return 3;
  if (!(rc > 0.0)) {
    if (m > 0) {
      // eq. csrc solved for r_c at the prescribed m (fixed point: c_s depends on r_c in abs mode)
      rc = L * std::log(1.0 / eps) / (kPi * m);
      for (int it = 0; it < 200; ++it) {
        const double r2 = L * cs_of(eps, L, rc, q_l2, tol_mode) / (kPi * m);
        const bool done = std::fabs(r2 - rc) <= 1e-15 * rc;
        rc = r2;
        if (done) break;
      }
    } else {
      if (n <= 0) return 1;
      rc = L * std::cbrt(3.0 * 64.0 / (4.0 * kPi * static_cast<double>(n)));  // 64 neighbours
    }
  }
  if (!(rc > 0.0) || !std::isfinite(rc)) return 1;
  const double cs = cs_of(eps, L, rc, q_l2, tol_mode);                       // Alg. 3 step 1
  const double Bw = as_over_aw() * std::sqrt(rc / L);
  const double arg = -2.0 * Bw * Bw * std::exp(-2.0 * cs) / cs;
  if (!(arg > -1.0 / std::exp(1.0) && arg < 0.0)) return 2;
  const double cw = -0.5 * lambert_wm1(arg);                                  // step 2
  const double alpha = rc * cw / cs;                                          // step 3
  const int m_alg = static_cast<int>(std::ceil(L * cs / (kPi * rc) - 1e-9));  // step 4
  int mm = m;
  if (mm > 0) {
    if (m_alg > mm) return 3;
  } else {
    mm = next_smooth_even(std::max(m_alg, 8));
    if (mm > 512) return 3;
  }
  const int P = static_cast<int>(std::ceil(2.0 * alpha * mm / L - 1e-9));     // step 5
  if (P < 2 || P > 32 || P > mm) return 3;
  const double h = L / mm;
  Params p{};
  p.L = L;
  p.eps = eps;
  p.rc = rc;
  p.cs = kPi * rc * mm / L;
  p.cw = kPi * P / 2.0;
  p.alpha = P * h / 2.0;
  p.h = h;
  p.cs_alg = cs;
  p.cw_alg = cw;
  p.alpha_alg = alpha;
  p.m = mm;
  p.P = P;
  p.tol_mode = tol_mode;
  if (p.cs > 40.0 || p.cw > 40.0) return 2;  // PSWF evaluation reaches machine precision (App. A)
  p.lambda0_s = Pswf(p.cs).lambda0;
  *out = p;
  return 0;
}

namespace {

// Chebyshev interpolation of f on [-1/2, 1/2] at deg+1 first-kind nodes, returned as monomial
// coefficients in g (long double throughout).
template <class F>
std::vector<long double> cheb_fit_monomial(F f, int deg) {
  const int N = deg + 1;
  std::vector<long double> fx(N), ck(N, 0.0L);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < N; ++i) {
    const long double th = pi * (i + 0.5L) / N;
    fx[i] = f(0.5L * std::cos(th));
  }
  for (int k = 0; k < N; ++k) {
    long double s = 0.0L;
    for (int i = 0; i < N; ++i) s += fx[i] * std::cos(pi * k * (i + 0.5L) / N);
    ck[k] = (k == 0 ? 1.0L : 2.0L) * s / N;
  }
  // sum_k ck T_k(2g): build T_k(2g) monomial coefficients by T_{k+1} = 4g T_k - T_{k-1}.
  std::vector<long double> out(N, 0.0L), t0(N, 0.0L), t1(N, 0.0L), t2(N, 0.0L);
  t0[0] = 1.0L;
  if (N > 1) t1[1] = 2.0L;
  for (int i = 0; i < N; ++i) out[i] += ck[0] * t0[i];
  if (N > 1)
    for (int i = 0; i < N; ++i) out[i] += ck[1] * t1[i];
  for (int k = 2; k < N; ++k) {
    for (int i = 0; i < N; ++i) t2[i] = (i > 0 ? 4.0L * t1[i - 1] : 0.0L) - t0[i];
    for (int i = 0; i < N; ++i) out[i] += ck[k] * t2[i];
    t0.swap(t1);
    t1.swap(t2);
  }
  return out;
}

}  // namespace

int choose_params_box(double eps, double Lx, double Ly, double Lz, double rc, int m, int64_t n, double q_l2,
                      int tol_mode, Params* out) {
  if (!out || !(Lx > 0.0) || !(Ly > 0.0) || !(Lz > 0.0) || !std::isfinite(Lx) || !std::isfinite(Ly) ||
      !std::isfinite(Lz))
    return 1;
  const double Lmin = std::min(Lx, std::min(Ly, Lz));
  const double ratio = Lmin * Lmin * Lmin / (Lx * Ly * Lz);  // volume of the cube / volume of the box
  const int64_t n_cube = n > 0 ? std::max<int64_t>(1, static_cast<int64_t>(std::llround(n * ratio))) : n;
  const int rcode = choose_params(eps, Lmin, rc, m, n_cube, q_l2 * std::sqrt(ratio), tol_mode, out);
  if (rcode != 0) return rcode;
  const double h = Lmin / out->m;
  const double Ls[3] = {Lx, Ly, Lz};
  int ms[3];
  for (int d = 0; d < 3; ++d) {
    ms[d] = next_smooth_even(static_cast<int>(std::ceil(Ls[d] / h - 1e-9)));
    if (ms[d] > 512) return 3;
  }
  out->L = Lx;
  out->Ly = Ly;
  out->Lz = Lz;
  out->m = ms[0];
  out->my = ms[1];
  out->mz = ms[2];
  out->h = Lx / ms[0];
  out->alpha = 0.5 * out->P * out->h;
  return 0;
}

int oversample_params(const Params& base, double sigma, Params* out) {
  if (!out || !(sigma >= 1.0) || sigma > 4.0 || base.split != kSplitPswf || base.window != kWindowPswf) return 1;
  Params p = base;
  double sig_eff = 1e300;
  for (int d = 0; d < 3; ++d) {
    const int md = next_smooth_even(static_cast<int>(std::ceil(sigma * base.grid(d) - 1e-9)));
    if (md > 512) return 3;
    (d == 0 ? p.m : (d == 1 ? p.my : p.mz)) = md;
    const double kband = base.cs * base.side(d) / (2.0 * kPi * base.rc);  // band edge in modes
    sig_eff = std::min(sig_eff, md / (2.0 * kband));
  }
  const double shrink = kPi * (1.0 - 1.0 / (2.0 * std::max(1.0, sig_eff)));
  const double cw_need = base.cw;  // the base grid's window bandlimit (pi P / 2 from Alg. 3)
  p.P = std::max(kPminHost, static_cast<int>(std::ceil(cw_need / shrink - 1e-9)));
  p.cw = shrink * p.P;
  p.h = p.L / p.m;
  p.alpha = 0.5 * p.P * p.h;
  p.alpha_alg = p.alpha;
  *out = p;
  return 0;
}

double default_gauss_shape(int P) { return 0.8 * kPi * P / 2.0; }

// Values M_{k+1}(t + r), r = 0..k, of the uniform B-spline of order k + 1 on [0, k + 1) at the
// points t + r, 0 <= t < 1, built up from M_1 = 1 on [0, 1) with
// M_{k+1}(y) = (y M_k(y) + (k + 1 - y) M_k(y - 1)) / k (the convolution with the unit box).
static void bspline_row(int order, long double t, long double* v) {
  v[0] = 1.0L;
  for (int k = 1; k < order; ++k) {
    v[k] = 0.0L;
    for (int r = k; r >= 0; --r) {
      const long double y = t + r;
      const long double a = r <= k - 1 ? y * v[r] : 0.0L;
      const long double b = r >= 1 ? (k + 1 - y) * v[r - 1] : 0.0L;
      v[r] = (a + b) / k;
    }
  }
}

long double bspline(int P, long double x) {
  const long double y = x + 0.5L * P;  // B_P(x) = M_P(x + P/2)
  if (!(y >= 0.0L && y < P)) return 0.0L;
  const int i = std::min(P - 1, static_cast<int>(std::floor(y)));
  long double v[64];
  bspline_row(P, y - i, v);
  return v[i];
}

long double bspline_deriv(int P, long double x) {
  // d/dy M_P(y) = M_{P-1}(y) - M_{P-1}(y - 1)
  const long double y = x + 0.5L * P;
  if (!(y >= 0.0L && y < P) || P < 2) return 0.0L;
  const int i = std::min(P - 1, static_cast<int>(std::floor(y)));
  long double v[64];
  bspline_row(P - 1, y - i, v);
  const long double a = i <= P - 2 ? v[i] : 0.0L;
  const long double b = i >= 1 ? v[i - 1] : 0.0L;
  return a - b;
}

void build_tables(const Params& p, int deg, double fit_tol, Tables* t) {
  const int m = p.m, P = p.P, half = m / 2;
  const double L = p.L, h = p.h, V = L * L * L;
  const bool gsplit = p.split == kSplitGauss;
  const Pswf ps(p.cs), pw(p.window == kWindowPswf ? p.cw : 1.0);
  const double sigma = p.rc / std::sqrt(p.cs);  // Gaussian split width, c_s = (r_c / sigma)^2
  // Radial part of the scaling, T_M[k2] = h^6 Mhat(k) / V with Mhat(k) = L^2 gammahat / (pi |k|^2)
  // (eq. Fsum). PSWF split: gammahat(w) = psi_0^{cs}(r_c w / c_s) / psi_0^{cs}(0) in band
  // (eq. PSWF_mollifier_ft), zero outside the band (|w| > c_s / r_c). Gaussian split (Example 1):
  // gammahat(w) = exp(-sigma^2 w^2 / 4) for |k| <= m/2. Zero at k = 0.
  const int k2max = 3 * half * half;
  const double kband = gsplit ? 0.5 * m : p.cs * L / (2.0 * kPi * p.rc);
  const double h6 = std::pow(h, 6);
  t->tm.assign(k2max + 1, 0.0);
  for (int k2 = 1; k2 <= k2max; ++k2) {
    const double k = std::sqrt(static_cast<double>(k2));
    if (k > kband * (1.0 + 1e-12)) continue;
    const double w = 2.0 * kPi * k / L;
    double gh;
    if (gsplit) {
      gh = std::exp(-0.25 * sigma * sigma * w * w);
    } else {
      const double s = std::min(1.0, p.rc * w / p.cs);
      gh = ps.psi(s) / ps.psi_0;
    }
    t->tm[k2] = h6 / V * L * L / (kPi * k2) * gh;
  }
  // Window factor W[k] = 1 / phihat_1(2 pi k / L)^2 (Table 2):
  //  PSWF: alpha lambda_0 psi(alpha w / c_w) / psi(0), with alpha w / c_w = 2k/m;
  //  Gaussian: the free-space transform alpha sqrt(pi / c_g) exp(-w^2 alpha^2 / (4 c_g));
  //  B-spline: h sum_j B_P(j) cos(2 pi k j / m), the periodised transform sum_p h B_P^(h w + 2 pi p)
  //  by Poisson summation (the SPME scaling).
  // One table per dimension d, with m_d, L_d, h_d = L_d / m_d and alpha_d = P h_d / 2 (on a
  // cuboid the window has the same P and c_w in grid units along every dimension).
  auto window_factors = [&](int d, std::vector<double>* out) {
    const int md = p.grid(d);
    const double Ld = p.side(d), hd = Ld / md, ad = 0.5 * P * hd;
    out->assign(md / 2 + 1, 0.0);
    for (int k = 0; k <= md / 2; ++k) {
      const double w = 2.0 * kPi * k / Ld;
      double ph = 0.0;
      if (p.window == kWindowPswf) {
        // alpha_d w / c_w = pi P k / (m_d c_w): 2k/m_d for c_w = pi P / 2, less on oversampled grids
        ph = ad * pw.lambda0 * pw.psi(std::min(1.0, kPi * P * k / (md * p.cw))) / pw.psi_0;
      } else if (p.window == kWindowGauss) {
        ph = ad * std::sqrt(kPi / p.cg) * std::exp(-w * w * ad * ad / (4.0 * p.cg));
      } else {
        long double acc = 0.0L;
        for (int j = -(P / 2); j <= P / 2; ++j)
          acc += bspline(P, static_cast<long double>(j)) * std::cos(2.0L * static_cast<long double>(kPi) * k * j / md);
        ph = hd * static_cast<double>(acc);
      }
      (*out)[k] = 1.0 / (ph * ph);
    }
  };
  window_factors(0, &t->w);
  window_factors(1, &t->wy);
  window_factors(2, &t->wz);
  // Cuboids: the radial factor is evaluated per mode on the GPU (|w|^2 is no integer function of
  // |k|^2 when the L_d / m_d or m_d differ).
  t->radial = 0;
  if (!p.cubic()) {
    const double hx = p.side(0) / p.grid(0), hy = p.side(1) / p.grid(1), hz = p.side(2) / p.grid(2);
    const double vol = p.side(0) * p.side(1) * p.side(2);
    t->rpref = 4.0 * kPi * hx * hx * hy * hy * hz * hz / vol;
    if (gsplit) {
      t->radial = 2;
      const double wmax = kPi / std::max(hx, std::max(hy, hz));  // |k_d| <= m_d / 2 on the coarsest axis
      t->rband2 = wmax * wmax;
      t->rsig2 = 0.25 * sigma * sigma;
    } else {
      t->radial = 1;
      t->rband2 = (p.cs / p.rc) * (p.cs / p.rc);
      t->rscale = (p.rc / p.cs) * (p.rc / p.cs);
      // psi_0(x) / psi_0(0) as a polynomial in u = x^2 - 1/2 on x in [0, 1]
      auto G = [&](long double u) -> long double {
        const double x = std::sqrt(std::max(0.0, std::min(1.0, static_cast<double>(u) + 0.5)));
        return static_cast<long double>(ps.psi(x) / ps.psi_0);
      };
      for (int dg = 8; dg <= 48; ++dg) {
        auto c = cheb_fit_monomial(G, dg);
        std::vector<double> coef(dg + 1);
        for (int k = 0; k <= dg; ++k) coef[k] = static_cast<double>(c[k]);
        double err = 0.0;
        for (int i = 0; i <= 256; ++i) {
          const double u = -0.5 + i / 256.0;
          double v = coef[dg];
          for (int k = dg - 1; k >= 0; --k) v = v * u + coef[k];
          err = std::max(err, std::fabs(v - static_cast<double>(G(u))));
        }
        t->rpoly.swap(coef);
        if (err <= 1e-15) break;
      }
    }
  }
  t->self_coef = gsplit ? 2.0 / (std::sqrt(kPi) * sigma) : 2.0 / (p.rc * ps.lambda0);
  // Piecewise-polynomial window (Remark after eq. force): one polynomial per support point, in
  // the offset g; the window at x = s alpha with s = 2 (g + (P-1)/2 - j) / P.
  auto window_at = [&](long double s) -> long double {
    s = std::max(-1.0L, std::min(1.0L, s));
    if (p.window == kWindowPswf) return static_cast<long double>(pw.psi(static_cast<double>(s)) / pw.psi_0);
    if (p.window == kWindowGauss) return std::exp(-static_cast<long double>(p.cg) * s * s);
    return bspline(P, 0.5L * P * s);  // x / h = s P / 2
  };
  auto window_ds = [&](long double s) -> long double {  // d/ds
    s = std::max(-1.0L, std::min(1.0L, s));
    if (p.window == kWindowPswf) return static_cast<long double>(pw.dpsi(static_cast<double>(s)) / pw.psi_0);
    if (p.window == kWindowGauss) return -2.0L * p.cg * s * std::exp(-static_cast<long double>(p.cg) * s * s);
    return 0.5L * P * bspline_deriv(P, 0.5L * P * s);
  };
  auto piece = [&](int j, long double g) -> long double {
    return window_at(2.0L * (g + 0.5L * (P - 1) - j) / P);
  };
  auto piece_d = [&](int j, double g) -> double {  // d/dg of phi_1(2(g + (P-1)/2 - j)/P)
    return static_cast<double>(window_ds(2.0L * (g + 0.5L * (P - 1) - j) / P) * 2.0L / P);
  };
  double dmax = 0.0;
  for (int j = 0; j < P; ++j)
    for (int i = 0; i <= 32; ++i) dmax = std::max(dmax, std::fabs(piece_d(j, -0.5 + i / 32.0)));
  const int dlo = deg > 0 ? deg : 4, dhi = deg > 0 ? deg : 28;
  for (int dg = dlo; dg <= dhi; ++dg) {
    std::vector<double> coef(static_cast<size_t>(P) * (dg + 1));
    for (int j = 0; j < P; ++j) {
      auto c = cheb_fit_monomial([&](long double g) { return piece(j, g); }, dg);
      for (int k = 0; k <= dg; ++k) coef[j * (dg + 1) + k] = static_cast<double>(c[k]);
    }
    double err = 0.0, derr = 0.0;
    for (int j = 0; j < P; ++j) {
      const double* c = &coef[j * (dg + 1)];
      for (int i = 0; i <= 96; ++i) {
        const double g = -0.5 + i / 96.0;
        double v = c[dg], dv = dg * c[dg];
        for (int k = dg - 1; k >= 0; --k) v = v * g + c[k];
        for (int k = dg - 1; k >= 1; --k) dv = dv * g + k * c[k];
        err = std::max(err, std::fabs(v - static_cast<double>(piece(j, g))));
        derr = std::max(derr, std::fabs(dv - piece_d(j, g)));
      }
    }
    t->deg = dg;
    t->coef.swap(coef);
    t->fit_err = err;
    t->fit_err_deriv = derr;
    if (err <= fit_tol && derr <= fit_tol * dmax) break;
  }
}

// The kernels evaluate the residual polynomial with at most this many powers in registers; the
// fit stops there (its sampled relative error reaches 1e-15 by degree 20 at every supported c_s,
// 1e-10 by degree 12 for c_s up to 16).
constexpr int kLocalMaxDeg = 24;

void build_local_table(const Params& p, double fit_tol, LocalTable* t) {
  const Pswf ps(p.cs);
  t->K = 2.0 / (ps.lambda0 * ps.psi_0 * p.rc);
  // G(t^2) = I(t) / t, with G(0) = psi_0(0)
  auto G = [&](long double g) -> long double {
    const double s = std::max(0.0, std::min(1.0, static_cast<double>(g) + 0.5));
    const double tt = std::sqrt(s);
    if (tt < 1e-8) return static_cast<long double>(ps.psi_0);
    return static_cast<long double>(ps.ipsi(tt) / tt);
  };
  const double gmax = static_cast<double>(G(-0.5L));
  for (int dg = 6; dg <= kLocalMaxDeg; ++dg) {
    auto c = cheb_fit_monomial(G, dg);
    std::vector<double> coef(dg + 1);
    for (int k = 0; k <= dg; ++k) coef[k] = static_cast<double>(c[k]);
    double err = 0.0;
    for (int i = 0; i <= 256; ++i) {
      const double g = -0.5 + i / 256.0;
      double v = coef[dg];
      for (int k = dg - 1; k >= 0; --k) v = v * g + coef[k];
      err = std::max(err, std::fabs(v - static_cast<double>(G(g))) / std::fabs(gmax));
    }
    t->deg = dg;
    t->coef.swap(coef);
    t->fit_err = err;
    if (err <= fit_tol) break;
  }
}

void twiddles(int N, int sign, std::vector<double>* out) {
  out->resize(2 * static_cast<size_t>(N));
  const long double twopi = 6.283185307179586476925286766559005768L;
  for (int e = 0; e < N; ++e) {
    const long double th = twopi * static_cast<long double>(e) / N;
    (*out)[2 * e] = static_cast<double>(std::cos(th));
    (*out)[2 * e + 1] = static_cast<double>(sign * std::sin(th));
  }
}

}  // namespace pswfe
