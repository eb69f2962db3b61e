"""C-ABI library checks that need no GPU: symbols, host-side float64 precompute against the
oracle (two independent implementations), and argument validation."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2602_16591_amd as pw
from conftest import ROOT
from oracle import fast, params as oparams
from oracle.pswf import PSWF, window_1d, window_1d_deriv

HEADER = os.path.join(ROOT, "include", "pswfe.h")


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pswfe_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pw.LIB_PATH)
    syms = header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(pw.SIGNATURES), "binding and header disagree"
    assert pw.version().startswith("pswfe")


@pytest.mark.parametrize("c", [1.0, 7.0, 13.8155, 18.85, 28.27, 35.0])
def test_host_pswf_matches_oracle(c):
    p = PSWF(c)
    for x in [0.0, 0.25, 0.6, 0.95, 1.0]:
        psi, dpsi, lam, chi = pw.host_pswf(c, x)
        assert abs(psi - p.psi(x)) < 1e-14 * p.psi_at_0
        assert abs(dpsi - p.dpsi(x)) < 1e-13 * max(1.0, c) * p.psi_at_0
        assert abs(lam - p.lambda0) < 1e-14
        assert abs(chi - p.chi0) < 1e-12 * max(1.0, p.chi0)


CASES = [
    dict(eps=1e-6, L=1.0, m=32, tol_mode="rel"),
    dict(eps=1e-6, L=6.688, m=64, tol_mode="rel"),
    dict(eps=1e-6, L=1.0, m=128, tol_mode="rel"),
    dict(eps=1e-10, L=1.0, rc=0.034370, tol_mode="rel"),
    dict(eps=1e-6, L=1.0, m=32, q_l2=31.6, tol_mode="abs"),
    dict(eps=1e-6, L=1.0, n=100000, tol_mode="rel"),
    dict(eps=1e-3, L=2.0, rc=0.3, tol_mode="rel"),
    dict(eps=1e-12, L=1.0, rc=0.1, q_l2=10.0, tol_mode="abs"),
]


@pytest.mark.parametrize("case", CASES)
def test_host_params_match_oracle(case):
    kw = dict(case)
    eps, L = kw.pop("eps"), kw.pop("L")
    c = pw.choose_params(eps, L, **kw).as_dict()
    o = oparams.choose(eps, L, **kw)
    assert (c["m"], c["P"]) == (o.m, o.P)
    for f in ["rc", "cs", "cw", "alpha", "cs_alg", "cw_alg", "alpha_alg"]:
        assert abs(c[f] - getattr(o, f)) <= 1e-12 * abs(getattr(o, f)), f
    assert abs(c["lambda0_s"] - PSWF(o.cs).lambda0) < 1e-14


@pytest.mark.parametrize("case", CASES[:5])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_host_tables_match_oracle(case, prec):
    """T_M[|k|^2] W[kx] W[ky] W[kz] equals the oracle's scaling s_k on the half spectrum, and the
    piecewise polynomials reproduce the window and its derivative within the fit tolerance."""
    kw = dict(case)
    eps, L = kw.pop("eps"), kw.pop("L")
    cp = pw.choose_params(eps, L, **kw)
    o = oparams.choose(eps, L, **kw)
    t = pw.host_tables(cp, prec)
    m, P = o.m, o.P
    s_or = fast.scaling(o, ball=True)
    k = fast.kvec(m)
    ak = np.abs(k)
    kx = np.arange(m // 2 + 1)
    k2 = kx[:, None, None] ** 2 + ak[None, :, None] ** 2 + ak[None, None, :] ** 2
    s_lib = t["tm"][k2] * t["w"][kx][:, None, None] * t["w"][ak][None, :, None] * t["w"][ak][None, None, :]
    s_ref = s_or[: m // 2 + 1, :, :]
    # psi_0(s) near s = 1 is ~eps_w psi_0(0) summed from O(1) Legendre terms, so both
    # implementations carry ~1e-16/eps_w relative rounding in 1/phihat^2 at the band edge; what
    # reaches the potential is s_k phihat(k)^2 (spreading and interpolation each multiply by phihat)
    phat2 = 1.0 / (t["w"][kx][:, None, None] * t["w"][ak][None, :, None] * t["w"][ak][None, None, :])
    assert np.max(np.abs(s_lib - s_ref) * phat2) <= 1e-12 * np.max(np.abs(s_ref) * phat2)
    assert np.array_equal(s_lib == 0, s_ref == 0)
    tol = max(0.01 * eps, 5e-9 if prec == "fp32" else 1e-15)
    assert t["fit_err"] <= tol
    pwf = PSWF(o.cw)
    g = np.linspace(-0.5, 0.5, 201)
    for j in range(P):
        s = 2 * (g + (P - 1) / 2 - j) / P
        v = np.polyval(t["coef"][j][::-1], g)
        dv = np.polyval(np.polyder(t["coef"][j][::-1]), g)
        assert np.max(np.abs(v - window_1d(s, pwf))) <= 1.5 * tol + 1e-16
        dref = window_1d_deriv(np.clip(s, -1, 1), pwf) * 2 / P
        assert np.max(np.abs(dv - dref)) <= 1.5 * tol * 4 + 1e-14
    assert abs(t["self_coef"] - 2 / (o.rc * PSWF(o.cs).lambda0)) < 1e-12 * t["self_coef"]


def test_status_codes():
    with pytest.raises(pw.PswfeError) as e:
        pw.choose_params(1e-20, 1.0, m=32)
    assert e.value.status == pw.E_EPS_RANGE
    with pytest.raises(pw.PswfeError) as e:
        pw.choose_params(1e-6, -1.0, m=32)
    assert e.value.status == pw.E_ARG
    with pytest.raises(pw.PswfeError) as e:
        pw.choose_params(1e-6, 1.0, m=33)
    assert e.value.status == pw.E_GRID
    with pytest.raises(pw.PswfeError) as e:
        pw.choose_params(1e-6, 1.0, m=16, rc=0.9)  # band needs m >= L c_s/(pi rc) = 5 -> ok; P > m fails
    with pytest.raises(pw.PswfeError) as e:
        pw.choose_params(1e-6, 1.0, tol_mode="abs", rc=0.1)  # abs mode needs ||q||
    assert e.value.status == pw.E_ARG
    p = pw.choose_params(1e-6, 1.0, m=32)
    lib = pw._lib()
    h = ctypes.c_void_p()
    assert lib.pswfe_plan_create(ctypes.byref(p), 7, 10, ctypes.byref(h)) == pw.E_PREC
    assert lib.pswfe_plan_create(ctypes.byref(p), 0, -1, ctypes.byref(h)) == pw.E_ARG
    bad = pw.CParams.from_buffer_copy(p)
    bad.m = 30 * 11
    assert lib.pswfe_plan_create(ctypes.byref(bad), 0, 10, ctypes.byref(h)) == pw.E_GRID
    assert lib.pswfe_compute(None, 0, None, None, None, None, None, None) == pw.E_ARG
    assert lib.pswfe_plan_destroy(None) == pw.OK
    # batch plans: argument checks happen before any device work
    arr = (pw.CParams * 2)(p, p)
    cnt = (ctypes.c_int64 * 2)(10, 20)
    assert lib.pswfe_batch_plan_create(0, arr, cnt, 0, None, ctypes.byref(h)) == pw.E_ARG
    assert lib.pswfe_batch_plan_create(2, arr, None, 0, None, ctypes.byref(h)) == pw.E_ARG
    assert lib.pswfe_batch_plan_create(2, arr, cnt, 7, None, ctypes.byref(h)) == pw.E_PREC
    assert lib.pswfe_batch_plan_create(2, (pw.CParams * 2)(p, bad), cnt, 0, None, ctypes.byref(h)) == pw.E_GRID
    assert lib.pswfe_batch_plan_create(2, arr, (ctypes.c_int64 * 2)(10, -1), 0, None, ctypes.byref(h)) == pw.E_ARG
    assert lib.pswfe_batch_plan_create(2, arr, (ctypes.c_int64 * 2)(2**30, 2**30), 0, None,
                                       ctypes.byref(h)) == pw.E_ARG
    assert lib.pswfe_batch_plan_create(2, arr, cnt, 0, (ctypes.c_int32 * 2)(8, 33), ctypes.byref(h)) == pw.E_ARG
    assert lib.pswfe_batch_compute(None, None, None, None, None, None, None) == pw.E_ARG
    assert lib.pswfe_batch_compute_grad(None, None, None, None, None, None, None) == pw.E_ARG
    assert lib.pswfe_plan_num_systems(None) == 0
    assert lib.pswfe_plan_system(None, 0, None, None, None, None) == pw.E_ARG
    for s in range(10):
        assert lib.pswfe_status_str(s) and lib.pswfe_status_str(s) != b"unknown status"
    assert (pw.E_NONNEUTRAL, pw.E_NONFINITE, pw.CHECK_INPUT) == (8, 9, 4)
    assert lib.pswfe_compute_ex(None, 0, None, None, None, None, None, 8, None) == pw.E_ARG


def test_tile_for_density():
    from paper_2602_16591_amd.autotune import tile_for_density
    # about `target` particles per tile: B^3 n / m^3 >= target with the smallest such B >= 4
    for m, n, t in [(16, 500, 256), (50, 20000, 128), (32, 32768, 64), (48, 1000, 4096), (24, 10**6, 32)]:
        b = tile_for_density(m, n, t)
        assert 4 <= b <= m
        if 4 < b < m:
            assert b ** 3 * n / m ** 3 >= t - 1e-9 and (b - 1) ** 3 * n / m ** 3 < t
    assert tile_for_density(16, 0, 256) == 8


@pytest.mark.parametrize("eps,m,L", [(1e-6, 32, 1.0), (1e-10, 48, 2.0), (1e-4, 20, 0.7), (1e-12, 64, 1.0)])
def test_host_residual_matches_oracle(eps, m, L):
    """The real-space residual the kernels evaluate, R(r) = (1 - Phi(r))/r (eq. R), and R'(r)/r,
    from the library's float64 fit, against the oracle's split function (Legendre series and
    its quadrature-free integral): relative to 1/r, and R(r_c) = 0 where Phi reaches 1."""
    from oracle import params as oparams
    from oracle.pswf import split_function, split_function_deriv
    c = pw.choose_params(eps, L, m=m)
    o = oparams.choose(eps, L, m=m)
    r = np.linspace(1e-4, 1.0, 4001) * o.rc
    R, dRr, info = pw.host_local(c, r)
    ps = PSWF(o.cs)
    Phi = split_function(r, o.rc, ps)
    Rref = (1.0 - Phi) / r
    dRref = (-split_function_deriv(r, o.rc, ps) / r - (1.0 - Phi) / r ** 2) / r
    assert info["fit_err"] <= 1e-15
    assert np.max(np.abs(R - Rref) * r) < 2e-15
    assert np.max(np.abs(dRr - dRref) * r ** 3) < 2e-12   # derivative of a degree <= 40 fit
    assert abs(pw.host_local(c, np.array([o.rc * (1 - 1e-12)]))[0][0]) < 1e-9 / o.rc
    assert pw.host_local(c, np.array([o.rc, 1.5 * o.rc, 0.0]))[0].tolist() == [0.0, 0.0, 0.0]
