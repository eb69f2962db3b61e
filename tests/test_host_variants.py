"""The library's host side for the comparison configurations (pswfe_variant_params, host
tables) against the oracle's definitions of the splits and windows (oracle/variants.py). CPU only:
these calls touch no GPU."""
import math

import numpy as np
import pytest

from oracle import variants as V

pw = pytest.importorskip("paper_2602_16591_amd")

CONFIGS = [
    # (split, window, m, P)
    ("pswf", "pswf", 42, 10),
    ("gauss", "pswf", 80, 10),
    ("gauss", "gauss", 80, 15),
    ("pswf", "gauss", 48, 9),
    ("pswf", "bspline", 64, 8),
    ("gauss", "bspline", 64, 7),
    ("pswf", "bspline", 48, 4),
    ("gauss", "bspline", 160, 24),
    ("gauss", "gauss", 128, 24),
]


@pytest.mark.parametrize("split,window,m,P", CONFIGS)
def test_host_tables_match_oracle(split, window, m, P):
    L, rc, cs = 1.0, 0.1, math.log(1e6)
    c = pw.variant_params(split, window, L, rc, cs, m, P, eps=1e-10)
    assert (c.split, c.window, c.m, c.P) == (pw.SPLITS[split], pw.WINDOWS[window], m, P)
    t = pw.host_tables(c, "fp64")
    vp = V.VariantParams(L, rc, cs, m, P, split=split, window=window, cg=c.cg)
    if window == "gauss":
        assert abs(c.cg - V.gauss_window_shape(P)) < 1e-12
    k = np.arange(m // 2 + 1)
    w_ref = 1.0 / V.window_hat(k, vp) ** 2
    # the PSWF window's 1/phihat^2 reaches e^{2 c_w} at the Nyquist mode; its two PSWF
    # evaluations (Legendre series here, Sturm + inverse iteration there) agree to ~1e-10
    assert np.max(np.abs(t["w"] - w_ref) / w_ref) < (1e-9 if window == "pswf" else 1e-11)
    kn = np.sqrt(np.arange(len(t["tm"]), dtype=np.float64))
    tm_ref = np.zeros(kn.size)
    tm_ref[1:] = (L / m) ** 6 * V.mhat(2 * math.pi * kn[1:] / L, vp) / L ** 3
    tm_ref[kn > V.band_edge(vp) * (1 + 1e-12)] = 0.0
    assert np.max(np.abs(t["tm"] - tm_ref)) < 1e-13 * np.max(np.abs(tm_ref))
    assert abs(t["self_coef"] - V.self_coefficient(vp)) < 1e-12 * V.self_coefficient(vp)
    # the piecewise polynomials reproduce the window on every piece
    g = np.linspace(-0.5, 0.5, 41)
    h = L / m
    for j in range(P):
        wv, _ = V.window_values((g + (P - 1) / 2 - j) * h, vp)
        assert np.max(np.abs(np.polyval(t["coef"][j][::-1], g) - wv)) < 1e-13
    if window == "bspline":
        assert t["deg"] <= max(4, P - 1)  # a B-spline piece is a polynomial of degree P - 1 (fits start at 4)


def test_variant_params_status_codes():
    ok = dict(split="gauss", window="bspline", L=1.0, rc=0.1, cs=10.0, m=32, P=6)
    pw.variant_params(**ok)
    for bad, status in [(dict(split=2), pw.E_ARG), (dict(window=5), pw.E_ARG),
                        (dict(L=-1.0), pw.E_ARG), (dict(rc=0.6), pw.E_ARG),
                        (dict(m=34), pw.E_GRID), (dict(P=2), pw.E_GRID), (dict(P=25), pw.E_GRID),
                        (dict(cs=41.0), pw.E_EPS_RANGE)]:
        with pytest.raises(pw.PswfeError) as ei:
            pw.variant_params(**{**ok, **bad})
        assert ei.value.status == status, bad
    # the residual exists for the PSWF split only
    c = pw.variant_params(**ok)
    with pytest.raises(pw.PswfeError) as ei:
        pw.host_local(c, np.array([0.05]))
    assert ei.value.status == pw.E_ARG
