"""Oversampled grids (oracle/variants.oversample; the paper leaves oversampling to future work):
with the window bandlimit set by the gap between the band edge and its first alias, a grid
finer than the band needs reaches the same tolerance with a smaller support; the library's rule
agrees with the oracle's."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct, params as oparams
from oracle import variants as V


@pytest.mark.parametrize("eps", [1e-6, 1e-10])
def test_oversampled_grid_meets_eps_with_smaller_support(eps):
    x, q, L = W.paper_default(100, seed=W.SEED_BASE)
    p = oparams.choose(eps, L, rc=0.1)
    ref, _ = direct.longrange_r2(x, q, L, p.rc, p.cs, grad=False)
    far = ref - direct.self_term(q, p.rc, p.cs)
    P_prev = p.P
    for sigma in (1.0, 1.5, 2.0):
        vp = V.oversample(p, sigma)
        if sigma == 1.0:
            assert (vp.m, vp.P) == (p.m, p.P) and abs(vp.cw - math.pi * p.P / 2) < 1e-12
        else:
            assert vp.P < P_prev or vp.P <= p.P - 2
        phi, _ = V.fast_variant(x, q, vp, grad=False)
        assert np.linalg.norm(phi - ref) / np.linalg.norm(far) <= eps, (sigma, vp.m, vp.P)
        P_prev = vp.P


def test_plain_window_bandlimit_gains_nothing_from_oversampling():
    """With c_w kept at pi P / 2 an oversampled grid does not allow a smaller support: the gain
    comes from the wider window band."""
    x, q, L = W.paper_default(100, seed=W.SEED_BASE)
    eps = 1e-6
    p = oparams.choose(eps, L, rc=0.1)
    ref, _ = direct.longrange_r2(x, q, L, p.rc, p.cs, grad=False)
    far = ref - direct.self_term(q, p.rc, p.cs)
    vp = V.oversample(p, 2.0)
    plain = V.VariantParams(vp.L, vp.rc, vp.cs, vp.m, vp.P)   # c_w = pi P / 2
    phi, _ = V.fast_variant(x, q, plain, grad=False)
    assert np.linalg.norm(phi - ref) / np.linalg.norm(far) > 3 * eps   # 9 eps here; the wider band gives 0.06 eps


def test_library_oversampling_matches_oracle():
    pw = pytest.importorskip("paper_2602_16591_amd")
    for eps, rc, sigma in [(1e-6, 0.1, 1.5), (1e-10, 0.1, 2.0), (1e-6, 0.15, 1.25), (1e-8, 0.12, 1.0)]:
        p = oparams.choose(eps, 1.0, rc=rc)
        vp = V.oversample(p, sigma)
        c = pw.oversample_params(pw.choose_params(eps, 1.0, rc=rc), sigma)
        assert (c.m, c.my, c.mz, c.P) == (vp.m, vp.m, vp.m, vp.P)
        assert abs(c.cw - vp.cw) < 1e-12 * vp.cw
    with pytest.raises(pw.PswfeError):
        pw.oversample_params(pw.choose_params(1e-6, 1.0, rc=0.1), 0.5)
