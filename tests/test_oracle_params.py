"""Pins of the oracle's parameter selection (oracle/params.py, Alg. 3)."""
import math

import numpy as np
import pytest

from oracle import params


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-10])
@pytest.mark.parametrize("rc", [0.05, 0.1, 0.2])
def test_alg3_abs_mode_plugs_back(eps, rc):
    """c_s solves the split model = eps (eq. cs_dimless from eq. PSWF_model); c_w balances the
    window model against the split model (eq. cwcs_model_dimless) with c_w > c_s/2 > 1/2."""
    L, qn = 1.0, 30.0
    p = params.choose(eps, L, rc=rc, q_l2=qn, tol_mode="abs")
    split = params.A_S * qn / math.sqrt(L ** 3) * math.sqrt(rc) * p.cs_alg ** -0.5 * math.exp(-p.cs_alg)
    assert abs(split / eps - 1) < 1e-10
    A_w = params.A_S / params.A_S_OVER_A_W
    lhs = math.sqrt(L) * A_w * math.sqrt(p.cw_alg) * math.exp(-p.cw_alg)
    rhs = math.sqrt(rc) * params.A_S / math.sqrt(p.cs_alg) * math.exp(-p.cs_alg)
    assert abs(lhs / rhs - 1) < 1e-10
    assert p.cw_alg > 0.5


@pytest.mark.parametrize("eps", [1e-2, 1e-6, 1e-12])
def test_alg3_rel_mode_and_rounding(eps):
    """c_s = log(1/eps); m = ceil(L c_s/(pi r_c)) rounded up to an even 2,3,5,7-smooth size;
    P = ceil(2 alpha m / L); the method then runs with c_s = pi r_c m / L, c_w = pi P/2,
    alpha = P h / 2, so c_w/alpha = c_s/r_c (eq. bandwidth) and c_w = pi P/2 (eq. cwP)."""
    L, rc = 2.0, 0.3
    p = params.choose(eps, L, rc=rc, tol_mode="rel")
    assert abs(p.cs_alg - math.log(1 / eps)) < 1e-14
    m_alg = math.ceil(L * p.cs_alg / (math.pi * rc))
    assert p.m >= m_alg and params.is_smooth_even(p.m)
    assert all(not params.is_smooth_even(k) for k in range(m_alg, p.m))
    assert p.P == math.ceil(2 * p.alpha_alg * p.m / L)
    assert abs(p.cs - math.pi * rc * p.m / L) < 1e-13
    assert abs(p.cw - math.pi * p.P / 2) < 1e-13
    assert abs(p.alpha - p.P * L / p.m / 2) < 1e-15
    assert abs(p.cw / p.alpha - p.cs / p.rc) < 1e-10 * p.cs / p.rc
    assert p.cs >= p.cs_alg and p.cw >= p.cw_alg - 1e-12


def test_prescribed_grid_solves_rc():
    """With m prescribed, r_c comes from eq. csrc (c_s/r_c = pi m / L) and m is kept."""
    for mode in ["rel", "abs"]:
        p = params.choose(1e-6, 1.0, m=32, q_l2=31.6, tol_mode=mode)
        assert p.m == 32
        assert abs(p.cs / p.rc - math.pi * 32) < 1e-9
        assert abs(p.cs - p.cs_alg) < 1e-9


def test_smooth_sizes():
    assert [k for k in range(2, 40) if params.is_smooth_even(k)] == \
        [2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 24, 28, 30, 32, 36]
    assert params.next_smooth_even(43) == 48 and params.next_smooth_even(211) == 216


def test_lambertw_branch_matters():
    """W_0 of the small negative argument would give c_w ~ 0 (no window); W_{-1} is the root
    of the balance with c_w > 1/2."""
    from scipy.special import lambertw
    Bw = params.A_S_OVER_A_W * math.sqrt(0.1)
    arg = -2 * Bw * Bw * math.exp(-2 * 13.8) / 13.8
    assert -0.5 * lambertw(arg, 0).real < 1e-10
    assert params.cw_from_cs(13.8, 0.1, 1.0) > 10.0
