"""Oracle: the first prolate spheroidal wave function of order zero, psi_0^c.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the paper's Sec. 2.5 and App. B:

* psi_0^c is the eigenfunction of the band-limited Fourier operator F_c (eq. operator,
  eq. eigenvalueproblem), L2-normalised on [-1, 1], even, with psi_0^c(0) > 0.
* On [-1, 1] it is expanded in even Legendre polynomials (eq. PSWFLegendre); substituting the
  expansion into the Sturm-Liouville equation (eq. ode) gives a symmetric tridiagonal
  eigenproblem whose smallest eigenvalue is chi_0 (App. B.1).
* lambda_0 = (1/psi_0(0)) int_{-1}^{1} psi_0 (App. B.3).
* psi_0' is the derivative of the Legendre series (App. B.4).

The tridiagonal matrix is written in the orthonormal basis  Pbar_n = sqrt(n + 1/2) P_n.
With  -((1 - x^2) P_n')' = n(n+1) P_n  and the three-term recurrence for x^2 P_n, the
operator  -((1-x^2) psi')' + c^2 x^2 psi  (whose eigenvalue is chi_0, eq. ode) has
  diagonal      n(n+1) + c^2 (2n(n+1) - 1) / ((2n+3)(2n-1))
  off-diagonal  c^2 (n+1)(n+2) / ((2n+3) sqrt((2n+1)(2n+5)))     between n and n+2.
The eigensolver is SciPy's ``eigh_tridiagonal`` (a library routine used as one step).

Pins (tests/test_oracle_pswf.py): Table 5 curve fits, Lemma 3 (chi_0 <= c^2/3), the bound
lambda_0 < sqrt(2 pi / c) (Sec. 2.5), Lemma 4 tail bound, the eigen-relation of Lemma 2
by independent quadrature, SciPy's spheroidal routines ``pro_cv``/``pro_ang1``, and the
c -> 0 limit (psi_0 -> 1/sqrt(2), lambda_0 -> 2).
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as _leg
from scipy.linalg import eigh_tridiagonal


def _n_terms(c: float) -> int:
    # App. B.5: K ~ 1.2 c terms suffice for 1e-12; a generous margin is taken here.
    return max(40, int(1.5 * c) + 30)


@functools.lru_cache(maxsize=256)
def _legendre_solution(c: float, K: int):
    n = 2.0 * np.arange(K)  # even degrees 0, 2, ..., 2K-2
    diag = n * (n + 1.0) + c * c * (2.0 * n * (n + 1.0) - 1.0) / ((2.0 * n + 3.0) * (2.0 * n - 1.0))
    m = n[:-1]
    off = c * c * (m + 1.0) * (m + 2.0) / ((2.0 * m + 3.0) * np.sqrt((2.0 * m + 1.0) * (2.0 * m + 5.0)))
    w, v = eigh_tridiagonal(diag, off, select="i", select_range=(0, 0))
    beta = v[:, 0]  # unit vector in the orthonormal basis -> ||psi||_{L2[-1,1]} = 1
    a = np.zeros(2 * K)
    a[0::2] = beta * np.sqrt(n + 0.5)  # coefficients in the standard Legendre basis P_n
    if _leg.legval(0.0, a) < 0.0:  # sign convention psi_0(0) > 0 (Sec. 2.5)
        a = -a
    return float(w[0]), a


class PSWF:
    """psi_0^c for one bandlimit c, evaluated from its Legendre expansion on [-1, 1]."""

    def __init__(self, c: float, K: int | None = None):
        self.c = float(c)
        self.K = _n_terms(self.c) if K is None else int(K)
        self.chi0, self.a = _legendre_solution(self.c, self.K)
        self.da = _leg.legder(self.a)
        self.ia = _leg.legint(self.a, lbnd=0.0)  # antiderivative vanishing at 0
        self.psi_at_0 = float(_leg.legval(0.0, self.a))
        self.psi_at_1 = float(_leg.legval(1.0, self.a))
        # App. B.3: lambda_0 = int_{-1}^{1} psi_0 / psi_0(0); int P_n = 0 for n > 0, = 2 for n = 0.
        self.lambda0 = 2.0 * self.a[0] / self.psi_at_0

    # --- values on [-1, 1] ---------------------------------------------------------------
    def psi(self, x):
        """psi_0^c(x) for |x| <= 1 (Legendre series, eq. PSWFLegendre)."""
        return _leg.legval(np.asarray(x, dtype=np.float64), self.a)

    def dpsi(self, x):
        """(psi_0^c)'(x) for |x| <= 1 (App. B.4, derivative of the series)."""
        return _leg.legval(np.asarray(x, dtype=np.float64), self.da)

    def ipsi(self, x):
        """int_0^x psi_0^c(u) du for |x| <= 1."""
        return _leg.legval(np.asarray(x, dtype=np.float64), self.ia)

    # --- values anywhere, from the eigen-relation ----------------------------------------
    def psi_ext(self, s, nquad: int | None = None):
        """psi_0^c(s) for any real s via eq. eigenvalueproblem:
        lambda_0 psi_0(s) = int_{-1}^{1} psi_0(t) e^{i c s t} dt  (psi_0 even -> cosine)."""
        s = np.asarray(s, dtype=np.float64)
        amax = self.c * float(np.max(np.abs(s))) if s.size else 0.0
        t, wq = _gauss(nquad or (2 * self.K + int(amax) + 64))
        f = self.psi(t)
        return (np.cos(self.c * np.multiply.outer(s, t)) @ (wq * f)) / self.lambda0


@functools.lru_cache(maxsize=64)
def _gauss(n: int):
    return np.polynomial.legendre.leggauss(n)


# ---------------------------------------------------------------------------------------
# Mollifier, split function and window (Sec. 4.2, 4.3)
# ---------------------------------------------------------------------------------------

def gammahat(omega, rc: float, pswf_s: PSWF, nquad: int | None = None):
    """Fourier transform of the PSWF mollifier gamma_{r_c}^{c_s} at |omega| (any omega).

    Defining integral (eq. gammahatintegral) with the 1/lambda_0 of the mollifier's
    normalisation (eq. PSWF_mollifier) written out:
        gammahat(w) = 1/(lambda_0 psi_0(0)) * int_{-1}^{1} psi_0(u) cos(w r_c u) du.
    Inside the band this equals psi_0(r_c w / c_s) / psi_0(0) (eq. PSWF_mollifier_ft).
    """
    omega = np.abs(np.asarray(omega, dtype=np.float64))
    amax = float(np.max(omega)) * rc if omega.size else 0.0
    t, wq = _gauss(nquad or (2 * pswf_s.K + int(amax) + 64))
    f = pswf_s.psi(t) * wq
    out = np.empty(omega.shape)
    flat = omega.reshape(-1)
    o = out.reshape(-1)
    step = 4096
    for i in range(0, flat.size, step):
        o[i:i + step] = np.cos(np.multiply.outer(flat[i:i + step] * rc, t)) @ f
    return out / (pswf_s.lambda0 * pswf_s.psi_at_0)


def split_function(r, rc: float, pswf_s: PSWF):
    """Phi_{r_c}^{c_s}(r) (eq. Phi_cs): 2/(lambda_0 psi_0(0)) int_0^{r/r_c} psi_0; 1 for r >= r_c."""
    r = np.asarray(r, dtype=np.float64)
    x = np.minimum(r / rc, 1.0)
    return 2.0 * pswf_s.ipsi(x) / (pswf_s.lambda0 * pswf_s.psi_at_0)


def split_function_deriv(r, rc: float, pswf_s: PSWF):
    """d/dr Phi_{r_c}(r) = 2 gamma_{r_c}(r) = 2 psi_0(r/r_c)/(r_c lambda_0 psi_0(0)), 0 beyond r_c."""
    r = np.asarray(r, dtype=np.float64)
    x = np.minimum(r / rc, 1.0)
    val = 2.0 * pswf_s.psi(x) / (rc * pswf_s.lambda0 * pswf_s.psi_at_0)
    return np.where(r < rc, val, 0.0)


def window_1d(s, pswf_w: PSWF):
    """phi_1^{c_w}(s) = psi_0(s)/psi_0(0) on [-1, 1], 0 outside (Sec. 4.3)."""
    s = np.asarray(s, dtype=np.float64)
    inside = np.abs(s) <= 1.0
    return np.where(inside, pswf_w.psi(np.clip(s, -1.0, 1.0)) / pswf_w.psi_at_0, 0.0)


def window_1d_deriv(s, pswf_w: PSWF):
    """d/ds phi_1^{c_w}(s) on [-1, 1] (Remark rem:force), 0 outside."""
    s = np.asarray(s, dtype=np.float64)
    inside = np.abs(s) <= 1.0
    return np.where(inside, pswf_w.dpsi(np.clip(s, -1.0, 1.0)) / pswf_w.psi_at_0, 0.0)


def window_hat_1d(omega, alpha: float, pswf_w: PSWF):
    """Fourier transform of the scaled 1-D window x -> phi_1(x/alpha) (Table 2):
    alpha lambda_0 psi_0(alpha omega / c_w) / psi_0(0), evaluated for |alpha omega| <= c_w."""
    s = np.abs(np.asarray(omega, dtype=np.float64)) * alpha / pswf_w.c
    if np.any(s > 1.0 + 1e-12):
        raise ValueError("window_hat_1d: argument outside the band")
    return alpha * pswf_w.lambda0 * pswf_w.psi(np.minimum(s, 1.0)) / pswf_w.psi_at_0
