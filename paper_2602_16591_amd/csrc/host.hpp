// Host-side float64 precompute for the PSWF fast Ewald plan: the PSWF itself (App. B),
// Lambert W, parameter selection (Alg. 3) and the tables the kernels read.
#pragma once

#include <cstdint>
#include <vector>

namespace pswfe {

// psi_0^c on [-1, 1] from its even Legendre expansion (eq. PSWFLegendre), with the
// Legendre coefficients from the smallest eigenpair of the symmetric tridiagonal matrix
// that the Sturm-Liouville equation (eq. ode) gives in the orthonormal Legendre basis,
// found by Sturm bisection and inverse iteration (App. B.2).
struct Pswf {
  double c = 0.0;
  double chi0 = 0.0;       // differential-equation eigenvalue (eq. ode)
  double lambda0 = 0.0;    // integral-operator eigenvalue (eq. eigenvalueproblem)
  double psi_0 = 0.0;      // psi_0^c(0)
  double psi_1 = 0.0;      // psi_0^c(1)
  std::vector<double> a;   // a[k]: coefficient of the Legendre polynomial P_{2k}

  explicit Pswf(double c);
  double psi(double x) const;   // |x| <= 1
  double dpsi(double x) const;  // |x| <= 1
  double ipsi(double x) const;  // int_0^x psi_0, |x| <= 1
};

double lambert_w0(double x);   // principal branch, x >= -1/e
double lambert_wm1(double x);  // lower branch, -1/e <= x < 0

// Kernel split and window (Sec. 4.2, 4.3; the comparison configurations of Sec. 4.3.1 and
// Sec. 7.3.1-7.4 use the Gaussian split of Example 1 and the Gaussian and B-spline windows of
// Table 2).
enum Split { kSplitPswf = 0, kSplitGauss = 1 };
enum Window { kWindowPswf = 0, kWindowGauss = 1, kWindowBspline = 2 };

struct Params {
  double L, eps, rc, cs, cw, alpha, h, lambda0_s;
  double cs_alg, cw_alg, alpha_alg;
  int m, P, tol_mode;
  int split = kSplitPswf;    // for the Gaussian split, cs = (rc / sigma)^2
  int window = kWindowPswf;
  double cg = 0.0;           // Gaussian window shape: exp(-cg (x/alpha)^2)
  // Cuboid boxes (Sec. 6.1): sides L (x), Ly, Lz and grid sizes m (x), my, mz; 0 means equal to
  // the x value. Grid spacings h_d = L_d / m_d; L, h and alpha above are the x values.
  double Ly = 0.0, Lz = 0.0;
  int my = 0, mz = 0;
  double side(int d) const { return d == 0 ? L : (d == 1 ? (Ly > 0 ? Ly : L) : (Lz > 0 ? Lz : L)); }
  int grid(int d) const { return d == 0 ? m : (d == 1 ? (my > 0 ? my : m) : (mz > 0 ? mz : m)); }
  bool cubic() const { return side(1) == L && side(2) == L && grid(1) == m && grid(2) == m; }
};

// Default Gaussian window shape for support P: 0.8 times c_w = pi P / 2 (the ratio that gave
// the smallest errors at the grid sizes and supports of Table 3's Gaussian/Gaussian column).
double default_gauss_shape(int P);

// Centred cardinal B-spline B_P(x) (Table 2) and its derivative, by the Cox-de Boor
// recurrence of the uniform spline on the piece that contains x.
long double bspline(int P, long double x);
long double bspline_deriv(int P, long double x);

bool is_smooth_even(int m);
int next_smooth_even(int m);

// Alg. 3 with the rounding rules documented in pswfe.h. Returns 0 on success, else a
// pswfe_status code.
int choose_params(double eps, double L, double rc, int m, int64_t n, double q_l2, int tol_mode,
                  Params* out);

// Alg. 3 for a cuboid box: the cube of side L_min with the same particle and charge densities
// fixes r_c, c_s, c_w, P and h = L_min / m; m_d is then the smallest even 2,3,5,7-smooth size
// with L_d / m_d <= h (Sec. 6.1, remark on cuboid domains).
int choose_params_box(double eps, double Lx, double Ly, double Lz, double rc, int m, int64_t n, double q_l2,
                      int tol_mode, Params* out);

// Oversampled grid (the paper leaves oversampling to future work; see the design notes): every
// m_d becomes the smallest FFT size >= sigma m_d, and with the effective factor
// sigma' = min_d m_d / (2 x band edge in modes) the PSWF window bandlimit is
// c_w = pi P (1 - 1/(2 sigma')), the distance from the band edge to its first alias in units of
// 1/alpha; P is the smallest support whose c_w reaches base's c_w (pi P / 2 from Alg. 3), so
// P shrinks by about 1 / (2 - 1/sigma'). sigma = 1 returns base's grid and support. PSWF split
// and window only; 1 <= sigma <= 4.
constexpr int kPminHost = 3;
int oversample_params(const Params& base, double sigma, Params* out);

// Tables consumed by the kernels, all float64.
struct Tables {
  // Scaling s_k = T_M[|k|^2] * W[|k_x|] * W[|k_y|] * W[|k_z|] (Alg. 2 step 3 with the h^6 of the
  // unnormalised DFT pair): T_M[k2] = h^6 Mhat(k) / V for 0 < |k| <= band edge, else 0 (the
  // PSWF split's band edge c_s L / (2 pi r_c); m/2 for the Gaussian split, which has no band);
  // W[k] = 1 / phihat_1(2 pi k / L)^2 for 0 <= k <= m/2, with phihat_1 the window's transform
  // (for the B-spline window, the SPME form: the transform of its integer samples).
  std::vector<double> tm;  // size 3 (m/2)^2 + 1 (cubes only)
  std::vector<double> w;   // size m/2 + 1
  std::vector<double> wy, wz;  // the window factors along y and z (my/2 + 1, mz/2 + 1)
  // Cuboids: the radial factor per mode, 4 pi prod_d h_d^2 / V * gammahat(|w|) / |w|^2 for
  // |w|^2 <= rband2, with gammahat the Gaussian exp(-rsig2 |w|^2) (radial 2) or, for the PSWF
  // split (radial 1), the polynomial rpoly in u = rscale |w|^2 - 1/2 (psi_0(r_c |w| / c_s) /
  // psi_0(0), fitted to 1e-15 relative).
  int radial = 0;
  std::vector<double> rpoly;
  double rscale = 0.0, rpref = 0.0, rband2 = 0.0, rsig2 = 0.0;
  // Piecewise-polynomial window: for support point j = 0..P-1 and centred offset
  // g in [-1/2, 1/2], phi_1(2 (g + (P-1)/2 - j) / P) ~ sum_k coef[j*(deg+1) + k] g^k, with
  // phi_1(s) the window at x = s alpha.
  int deg = 0;
  std::vector<double> coef;     // P * (deg + 1)
  double fit_err = 0.0;         // max |fit - phi_1| over all pieces (sampled)
  double fit_err_deriv = 0.0;   // max |fit' - d phi_1/dg| over all pieces (sampled)
  double self_coef = 0.0;       // lim_{r->0} M(r): 2 / (rc lambda_0(c_s)), or 2 / (sqrt(pi) sigma)
};

// deg <= 0 picks the smallest degree in [4, 28] whose sampled error is below `fit_tol`.
void build_tables(const Params& p, int deg, double fit_tol, Tables* t);

// Real-space residual R(r) = (1 - Phi(r)) / r for r < r_c (Sec. 3.1.1, eq. R). With
// Phi(r) = 2 I(r/r_c) / (lambda_0 psi_0(0)), I(t) = int_0^t psi_0 (eq. Phi_cs), the smooth part
// M(r) = Phi(r)/r = K G(r^2/r_c^2) with K = 2 / (lambda_0 psi_0(0) r_c) and G(t^2) = I(t)/t,
// an even function of t. G is fitted as a polynomial in g = r^2/r_c^2 - 1/2 on [-1/2, 1/2].
struct LocalTable {
  int deg = 0;
  std::vector<double> coef;  // deg + 1 monomial coefficients in g
  double K = 0.0;
  double fit_err = 0.0;      // max |fit - G| / max |G| (sampled)
};
// Fits G to relative accuracy fit_tol (the lowest degree from 6 up that reaches it, at most 24).
void build_local_table(const Params& p, double fit_tol, LocalTable* t);

// exp(sign * 2 pi i e / N) for e = 0..N-1, as interleaved (re, im) pairs, float64.
void twiddles(int N, int sign, std::vector<double>* out);

}  // namespace pswfe
