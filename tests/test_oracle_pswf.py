"""Pins of the oracle's PSWF (oracle/pswf.py) against what the paper and mathematics fix.

Each check would fail for a plausible mistake in the tridiagonal matrix (wrong diagonal or
off-diagonal term, wrong basis scaling), the sign/normalisation convention, or lambda_0.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import pro_ang1, pro_cv, spherical_jn

from conftest import read_table
from oracle.pswf import PSWF, gammahat, split_function, split_function_deriv

CS = [7.0, 10.0, 14.0, 20.0, 28.0, 35.0]


# Table 5 states max relative errors of 1.6% (psi_0(1)) and 1.5% (ratio) for its endpoint fits,
# but the true values drift from the rounded fits by up to 4% over 7 <= c <= 35 (the ratio is
# normalisation-free and matches SciPy's independent pro_ang1 to ~1e-7, see the test below).
# The endpoint fits are therefore pinned with a 4.5% band; lambda_0 and psi_0(0) at the printed
# bounds (plus a 25% margin for the 3-4 digit rounding of the fit constants).
ENDPOINT_BAND = 0.045


@pytest.mark.parametrize("c", CS)
def test_table5_curve_fits(c):
    """Table 5 (App. A): fitted models on 7 <= c <= 35."""
    p = PSWF(c)
    fits = {r[0]: (r[1], float(r[2])) for r in read_table("table5_fits.txt")}
    got = {"lambda0": p.lambda0, "psi0_at_0": p.psi_at_0, "psi0_at_1": p.psi_at_1,
           "ratio_1_over_0": p.psi_at_1 / p.psi_at_0}
    for name, (expr, tol) in fits.items():
        model = eval(expr, {"c": c, "sqrt": math.sqrt, "exp": math.exp, "pi": math.pi})
        bound = ENDPOINT_BAND if name in ("psi0_at_1", "ratio_1_over_0") else 1.25 * tol
        assert abs(got[name] / model - 1.0) <= bound, (name, got[name], model)


@pytest.mark.parametrize("c", [7.0, 14.0, 20.0])
def test_endpoint_ratio_matches_scipy(c):
    """psi_0(1)/psi_0(0) (the eps_w of the window) against SciPy's prolate angular function."""
    p = PSWF(c)
    s1 = pro_ang1(0, 0, c, 1.0 - 1e-9)[0] / pro_ang1(0, 0, c, 0.0)[0]
    assert abs(p.psi_at_1 / p.psi_at_0 / s1 - 1.0) < 1e-5


@pytest.mark.parametrize("c", [0.5, 1.0, math.sqrt(3.0)] + CS)
def test_chi0_matches_scipy_and_lemma3(c):
    """chi_0 equals the spheroidal eigenvalue of SciPy's pro_cv and obeys Lemma 3 (chi_0 <= c^2/3)."""
    p = PSWF(c)
    assert abs(p.chi0 - pro_cv(0, 0, c)) <= 1e-10 * max(1.0, p.chi0)
    assert p.chi0 <= c * c / 3.0 + 1e-12


@pytest.mark.parametrize("c", [1.0, 5.0] + CS)
def test_lambda0_bound(c):
    """Sec. 2.5: sqrt(2 pi / c) > |lambda_0(c)| (equal to rounding once e^{-2c} < 1e-16)."""
    assert PSWF(c).lambda0 <= math.sqrt(2.0 * math.pi / c) * (1 + 4e-16)


def test_fuchs_asymptotic():
    """App. A, eq. fuchs: 1 - mu_0(c) ~ 4 sqrt(pi c) e^{-2c} with mu_0 = c lambda_0^2 / (2 pi); the
    ratio approaches 1 from below as c grows."""
    ratios = []
    for c in [5.0, 7.0, 9.0, 11.0, 13.0]:
        p = PSWF(c)
        one_minus_mu = 1.0 - c * p.lambda0 ** 2 / (2 * math.pi)
        ratios.append(one_minus_mu / (4 * math.sqrt(math.pi * c) * math.exp(-2 * c)))
    assert all(0.88 < r < 1.0 for r in ratios)
    assert all(b > a for a, b in zip(ratios, ratios[1:]))


@pytest.mark.parametrize("c", [2.0, 7.0, 20.0])
def test_shape_matches_scipy_angular_function(c):
    """psi_0(x)/psi_0(0) equals the ratio of SciPy's prolate angular function S_00(c, x)."""
    p = PSWF(c)
    x = np.linspace(-0.99, 0.99, 23)
    s = np.array([pro_ang1(0, 0, c, xi)[0] for xi in x])
    s0 = pro_ang1(0, 0, c, 0.0)[0]
    np.testing.assert_allclose(p.psi(x) / p.psi_at_0, s / s0, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("c", [1.0, 10.0, 30.0])
def test_normalisation_and_sign(c):
    """||psi_0||_{L2[-1,1]} = 1, psi_0 even, psi_0(0) > 0, psi_0 > 0 on (-1, 1) (Sec. 2.5)."""
    p = PSWF(c)
    val, _ = integrate.quad(lambda t: float(p.psi(t)) ** 2, -1, 1, limit=200, epsabs=1e-14)
    assert abs(val - 1.0) < 1e-10
    x = np.linspace(-1, 1, 401)
    assert p.psi_at_0 > 0
    assert np.all(p.psi(x[1:-1]) > 0)
    np.testing.assert_allclose(p.psi(x), p.psi(-x), rtol=0, atol=1e-14)


@pytest.mark.parametrize("c", [3.0, 15.0, 30.0])
def test_ode_residual(c):
    """psi_0 solves (1-s^2) psi'' - 2 s psi' + (chi_0 - c^2 s^2) psi = 0 (eq. ode)."""
    from numpy.polynomial import legendre as lg
    p = PSWF(c)
    s = np.linspace(-0.95, 0.95, 41)
    d1 = lg.legval(s, lg.legder(p.a))
    d2 = lg.legval(s, lg.legder(p.a, 2))
    res = (1 - s * s) * d2 - 2 * s * d1 + (p.chi0 - c * c * s * s) * p.psi(s)
    scale = c * c * np.max(np.abs(p.psi(s)))
    assert np.max(np.abs(res)) < 1e-9 * scale


@pytest.mark.parametrize("c", [2.0, 12.0, 25.0])
def test_eigen_relation_lemma2(c):
    """Lemma 2 / eq. eigenvalueproblem: int_{-1}^{1} psi_0(t) e^{icst} dt = lambda_0 psi_0(s), by
    adaptive quadrature (independent of the Gauss-Legendre rule used in the oracle)."""
    p = PSWF(c)
    for s in [0.0, 0.3, 0.77, 1.0]:
        val, _ = integrate.quad(lambda t: float(p.psi(t)) * math.cos(c * s * t), -1, 1,
                                limit=400, epsabs=1e-15, epsrel=1e-13)
        assert abs(val - p.lambda0 * float(p.psi(s))) < 1e-11 * p.lambda0 * p.psi_at_0


@pytest.mark.parametrize("c", [math.sqrt(3.0), 5.0, 10.0, 20.0])
def test_tail_bound_lemma4(c):
    """Lemma 4: |psi_0(s)| <= psi_0(1)/s for s >= 1 and c >= sqrt(3); and psi_ext agrees with the
    series on [-1, 1]."""
    p = PSWF(c)
    s = np.linspace(1.0, 12.0, 600)
    tail = p.psi_ext(s)
    assert np.all(np.abs(tail) <= p.psi_at_1 / s * (1 + 1e-9) + 1e-15)
    x = np.linspace(-1, 1, 21)
    np.testing.assert_allclose(p.psi_ext(x), p.psi(x), rtol=1e-11, atol=1e-14)


def test_small_c_limit():
    """c -> 0: F_c tends to integration against 1, psi_0 -> 1/sqrt(2), lambda_0 -> 2."""
    p = PSWF(1e-4)
    assert abs(p.psi_at_0 - 1 / math.sqrt(2)) < 1e-8
    assert abs(p.lambda0 - 2.0) < 1e-8


@pytest.mark.parametrize("c,rc", [(8.0, 0.2), (14.0, 0.13), (30.0, 0.05)])
def test_gammahat(c, rc):
    """Mollifier transform: gammahat(0) = 1 (unit mass); in band it equals
    psi_0(r_c w/c)/psi_0(0) (eq. PSWF_mollifier_ft); everywhere it equals the spherical-Bessel
    series 2 sum a_n (-1)^{n/2} j_n(w r_c)/(lambda_0 psi_0(0)) and direct adaptive quadrature
    of the real-space mollifier (eq. PSWF_mollifier)."""
    p = PSWF(c)
    assert abs(gammahat(0.0, rc, p) - 1.0) < 1e-13
    w = np.linspace(0, c / rc, 50)
    np.testing.assert_allclose(gammahat(w, rc, p), p.psi(rc * w / c) / p.psi_at_0, rtol=0, atol=1e-13)
    w2 = np.linspace(0, 4 * c / rc, 37)
    n = np.arange(p.a.size)
    series = np.array([np.sum(p.a[0::2] * 2.0 * (-1.0) ** (n[0::2] // 2) * spherical_jn(n[0::2], wi * rc))
                       for wi in w2]) / (p.lambda0 * p.psi_at_0)
    np.testing.assert_allclose(gammahat(w2, rc, p), series, rtol=0, atol=1e-13)
    for wi in [0.7 * c / rc, 1.9 * c / rc]:
        val, _ = integrate.quad(lambda x: float(p.psi(x / rc)) / (rc * p.lambda0 * p.psi_at_0) * math.cos(wi * x),
                                -rc, rc, limit=400, epsabs=1e-15)
        assert abs(val - gammahat(wi, rc, p)) < 1e-12


@pytest.mark.parametrize("c", [1.0, 6.0, 21.0, 49.0 / 1.4])
def test_split_function(c):
    """Sec. 4.1 and Fig. 3: Phi(r_c) = 1 so R(r >= r_c) = 0; 0 <= Phi <= 1, Phi nondecreasing;
    R >= 0; dPhi/dr = 2 gamma_{r_c} (checked by finite differences)."""
    rc = 0.5
    p = PSWF(c)
    r = np.linspace(0, rc, 501)
    Phi = split_function(r, rc, p)
    assert abs(Phi[-1] - 1.0) < 1e-13
    assert np.all(Phi >= -1e-15) and np.all(Phi <= 1 + 1e-13)
    assert np.all(np.diff(Phi) >= -1e-15)
    R = (1 - Phi[1:]) / r[1:]
    assert np.all(R >= -1e-13)
    np.testing.assert_allclose(split_function(np.array([rc, 1.3 * rc, 5.0]), rc, p), 1.0, rtol=0, atol=1e-13)
    h = 1e-6
    rr = np.linspace(0.01, 0.49, 13)
    fd = (split_function(rr + h, rc, p) - split_function(rr - h, rc, p)) / (2 * h)
    np.testing.assert_allclose(fd, split_function_deriv(rr, rc, p), rtol=1e-7, atol=1e-9)
