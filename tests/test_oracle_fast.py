"""Pins of the oracle's fast method (oracle/fast.py, Alg. 2) against the paper's printed
resolution table, its error models, and exact identities of the algorithm."""
import math

import numpy as np
import pytest

import workloads as W
from conftest import read_table
from oracle import direct, fast, params
from oracle.params import Params


def _params(L, rc, cs, m, P, eps=1e-6):
    h = L / m
    return Params(L=L, eps=eps, tol_mode="rel", rc=rc, cs=cs, cw=math.pi * P / 2, alpha=P * h / 2,
                  m=m, P=P, cs_alg=cs, cw_alg=math.pi * P / 2, alpha_alg=P * h / 2)


@pytest.mark.slow
def test_table3_pp_column():
    """Table 3 (PP): with n = 100, N(0,1) neutral charges, L = 1, r_c = 0.1, c_s = log(1/eps),
    the smallest m (at P+1) and the smallest P (at the paper's m) reaching relative l2 <= eps
    agree with the printed values (m within 1, P within 2; the workload is a random draw)."""
    x, q, L = W.paper_default(100, seed=W.SEED_BASE)
    rc = 0.1
    for row in read_table("table3_pp.txt"):
        eps, m_pap, P_pap = float(row[0]), int(row[1]), int(row[2])
        cs = math.log(1 / eps)
        ref, _ = direct.longrange_r2(x, q, L, rc, cs, grad=False)
        far = ref - direct.self_term(q, rc, cs)

        def err(m, P):
            ph, _ = fast.fast_longrange(x, q, _params(L, rc, cs, m, P), grad=False)
            return np.linalg.norm(ph - ref) / np.linalg.norm(far)

        m_min = next(m for m in range(m_pap - 3, m_pap + 4) if err(m, P_pap + 1) <= eps)
        P_min = next(P for P in range(P_pap - 4, P_pap + 5) if err(m_pap, P) <= eps)
        assert abs(m_min - m_pap) <= 1, (eps, m_min, m_pap)
        assert abs(P_min - P_pap) <= 2, (eps, P_min, P_pap)


@pytest.mark.parametrize("n,rc,seed", [(100, 0.1, 1), (600, 0.15, 2)])
def test_error_tracks_tolerance_abs_mode(n, rc, seed):
    """Fig. 8 / Alg. 3: with the absolute-RMS parameter choice the measured absolute RMS error
    of phi is close to, and not above, the requested eps."""
    x, q, L = W.paper_default(n, seed=seed)
    for eps in [1e-3, 1e-6, 1e-9]:
        p = params.choose(eps, L, rc=rc, q_l2=np.linalg.norm(q), tol_mode="abs")
        ref, _ = direct.longrange_r2(x, q, L, p.rc, p.cs, grad=False)
        ph, _ = fast.fast_longrange(x, q, p, grad=False)
        ratio = np.sqrt(np.mean((ph - ref) ** 2)) / eps
        assert 0.03 < ratio < 1.5, (eps, ratio)


def test_rel_mode_meets_eps_on_plain_config():
    """n = 1000 uniform +-1 charges, L = 1, eps = 1e-6 (relative mode), grid 32^3: relative l2
    error of phi_far against the direct sum is below eps; cube truncation (no band limit on
    the modes) is worse."""
    x, q, L = W.config("plain_fp64_n1000")
    p = params.choose(1e-6, L, m=32, tol_mode="rel")
    ref, _ = direct.longrange_r2(x, q, L, p.rc, p.cs, grad=False)
    far = ref - direct.self_term(q, p.rc, p.cs)
    ph, _ = fast.fast_longrange(x, q, p, grad=False)
    assert np.linalg.norm(ph - ref) / np.linalg.norm(far) < 1e-6
    ph_cube, _ = fast.fast_longrange(x, q, p, ball=False, grad=False)
    assert np.linalg.norm(ph_cube - ref) > np.linalg.norm(ph - ref)


def test_model_plateaus_fig5():
    """Fig. 5: at generous P the error sits on the split-error model (eq. PSWF_model), at
    generous m on the window-error model (eq. window_err_model), within a factor 3."""
    x, q, L = W.paper_default(100, seed=W.SEED_BASE)
    rc, qn = 0.1, np.linalg.norm(q)
    m = 40
    cs = math.pi * rc * m / L
    ref, _ = direct.longrange_r2(x, q, L, rc, cs, grad=False)
    ph, _ = fast.fast_longrange(x, q, _params(L, rc, cs, m, 16), grad=False)
    e_split = np.sqrt(np.mean((ph - ref) ** 2))
    model_s = params.A_S * qn * math.sqrt(rc) * cs ** -0.5 * math.exp(-cs)
    assert 1 / 3 < e_split / model_s < 3
    m2, P = 64, 7
    cs2 = math.pi * rc * m2 / L
    ref2, _ = direct.longrange_r2(x, q, L, rc, cs2, grad=False)
    ph2, _ = fast.fast_longrange(x, q, _params(L, rc, cs2, m2, P), grad=False)
    e_win = np.sqrt(np.mean((ph2 - ref2) ** 2))
    cw = math.pi * P / 2
    model_w = params.A_S / params.A_S_OVER_A_W * qn * math.sqrt(L) * cw ** 0.5 * math.exp(-cw)
    assert 1 / 3 < e_win / model_w < 3


def test_energy_identity():
    """Particle-side and grid-side energies agree: 1/2 sum rho_i phi_far,i = 1/2 sum_k s_k |ahat_k|^2
    (the scaling is real and even, so S^T F^-1 C D F S is a symmetric quadratic form, eq. matform)."""
    x, q, L = W.uniform_pm1(300, seed=4, L=1.7)
    p = params.choose(1e-6, L, m=24, tol_mode="rel")
    ph, _, gr = fast.fast_longrange(x, q, p, grad=False, return_grids=True)
    far = ph - direct.self_term(q, p.rc, p.cs)
    e_part = 0.5 * np.dot(q, far)
    e_grid = 0.5 * np.sum(gr["s"] * np.abs(gr["ahat"]) ** 2)
    assert abs(e_part - e_grid) < 1e-11 * abs(e_grid)


def test_forces_are_gradient_of_fast_energy():
    """The interpolated gradient (eq. force) is the exact position derivative of the fast
    method's own energy, away from stencil shifts (where the window value psi_0(1)/psi_0(0)
    at the support edge makes the energy jump by ~eps_w)."""
    x, q, L = W.uniform_pm1(200, seed=8)
    p = params.choose(1e-8, L, m=30, tol_mode="rel")
    ph, g = fast.fast_longrange(x, q, p)

    def energy(xx):
        pp, _ = fast.fast_longrange(xx, q, p, grad=False)
        return 0.5 * np.dot(q, pp)

    hstep = 1e-6
    checked = 0
    for i in range(0, 200, 17):
        for d in range(3):
            t = x[i, d] / p.h - p.P / 2
            if min(t - math.floor(t), math.ceil(t) - t) < 10 * hstep / p.h:
                continue
            xp, xm = x.copy(), x.copy()
            xp[i, d] += hstep
            xm[i, d] -= hstep
            fd = (energy(xp) - energy(xm)) / (2 * hstep)
            assert abs(fd - q[i] * g[i, d]) < 1e-6 * np.max(np.abs(q[:, None] * g)), (i, d)
            checked += 1
    assert checked > 20
