"""GPU parity of the comparison configurations (Sec. 4.3.1, Sec. 7.3.1-7.4): the Gaussian split
and the Gaussian and B-spline windows run through the same HIP kernels as the PSWF method, checked
element by element against the float64 oracle's Alg. 2 with the same split and window
(oracle/variants.py), and against the split's direct Fourier sum at the paper's resolutions."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct
from oracle import variants as V

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pw = pytest.importorskip("paper_2602_16591_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def tdev(a, prec):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32 if prec == "fp32" else torch.float64,
                           device=dev())


def fit_tol(eps, prec):
    return max(0.01 * eps, 5e-9 if prec == "fp32" else 1e-15)


CASES = [
    # (name, split, window, eps, m, P): Table 3 / Table 4 settings, m rounded up to an FFT size
    ("GG_1e-6", "gauss", "gauss", 1e-6, 80, 15),
    ("GP_1e-6", "gauss", "pswf", 1e-6, 80, 10),
    ("PB_P8_1e-5", "pswf", "bspline", 1e-5, 50, 8),
    ("GB_P6_1e-5", "gauss", "bspline", 1e-5, 108, 6),
    ("PB_P4_1e-4", "pswf", "bspline", 1e-4, 80, 4),
    ("GB_P5_odd", "gauss", "bspline", 1e-4, 64, 5),
    ("PG_mixed", "pswf", "gauss", 1e-6, 48, 12),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_variant_matches_oracle(case, prec):
    _, split, window, eps, m, P = case
    x, q, L = W.paper_default(1500, seed=61)
    if prec == "fp32":
        x, q = x.astype(np.float32).astype(np.float64), q.astype(np.float32).astype(np.float64)
    rc, cs = 0.1, math.log(1.0 / eps)
    c = pw.variant_params(split, window, L, rc, cs, m, P, eps=eps)
    vp = V.VariantParams(L, rc, cs, m, P, split=split, window=window, cg=c.cg)
    plan = pw.Plan(c, prec, n_max=len(q))
    phi, F, E = plan.compute(tdev(x, prec), tdev(q, prec))
    rphi, rg = V.fast_variant(x, q, vp)
    far = rphi + V.self_coefficient(vp) * q
    tol_phi = (1e-11 if prec == "fp64" else 2e-6) + 10 * fit_tol(eps, prec)
    tol_F = (1e-10 if prec == "fp64" else 2e-5) + 100 * fit_tol(eps, prec)
    phi = phi.double().cpu().numpy()
    assert np.linalg.norm(phi - rphi) / np.linalg.norm(far) < tol_phi
    rF = direct.forces(q, rg)
    assert np.linalg.norm(F.double().cpu().numpy() - rF) / np.linalg.norm(rF) < tol_F
    Eref = 0.5 * float(q @ rphi)
    assert abs(float(E.cpu()[0]) - Eref) <= tol_phi * 0.5 * float(np.abs(q) @ np.abs(far)) + 1e-12 * abs(Eref)


@pytest.mark.parametrize("case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_variant_accuracy_vs_direct_sum(case):
    """At these resolutions the float64 GPU result is within 2.5 eps (relative l2 of phi_far) of
    the split's own direct Fourier sum, as the paper's tables state for its settings."""
    _, split, window, eps, m, P = case
    x, q, L = W.paper_default(100, seed=W.SEED_BASE)
    rc, cs = 0.1, math.log(1.0 / eps)
    c = pw.variant_params(split, window, L, rc, cs, m, P, eps=eps)
    vp = V.VariantParams(L, rc, cs, m, P, split=split, window=window, cg=c.cg)
    if split == "pswf":
        ref, _ = direct.longrange_r2(x, q, L, rc, cs, grad=False)
    else:
        ref, _ = V.far_direct_variant(x, q, vp, V.reference_modes(vp))
    plan = pw.Plan(c, "fp64", n_max=len(q))
    phi, _, _ = plan.compute(tdev(x, "fp64"), tdev(q, "fp64"), force=False, energy=False)
    err = np.linalg.norm(phi.cpu().numpy() - ref) / np.linalg.norm(ref + V.self_coefficient(vp) * q)
    assert err <= 2.5 * eps, err / eps


def test_gaussian_split_has_no_residual():
    x, q, L = W.paper_default(100, seed=62)
    c = pw.variant_params("gauss", "gauss", L, 0.1, 10.0, 32, 8)
    plan = pw.Plan(c, "fp64", n_max=len(q))
    with pytest.raises(pw.PswfeError) as ei:
        plan.compute(tdev(x, "fp64"), tdev(q, "fp64"), total=True)
    assert ei.value.status == pw.E_ARG


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("sigma", [1.5, 2.0])
def test_oversampled_grid_matches_oracle(sigma, prec):
    """A grid oversampled by sigma with the smaller support it allows (pswfe_oversample_params):
    element-wise parity with the oracle's Alg. 2 on the same parameters, and the tolerance met
    against the direct sum."""
    from oracle import params as oparams
    eps = 1e-6
    x, q, L = W.paper_default(1500, seed=63)
    if prec == "fp32":
        x, q = x.astype(np.float32).astype(np.float64), q.astype(np.float32).astype(np.float64)
    c = pw.oversample_params(pw.choose_params(eps, L, rc=0.1), sigma)
    vp = V.oversample(oparams.choose(eps, L, rc=0.1), sigma)
    assert (c.m, c.P) == (vp.m, vp.P) and abs(c.cw - vp.cw) < 1e-12 * vp.cw
    plan = pw.Plan(c, prec, n_max=len(q))
    phi, F, _ = plan.compute(tdev(x, prec), tdev(q, prec))
    rphi, rg = V.fast_variant(x, q, vp)
    far = rphi + V.self_coefficient(vp) * q
    tol_phi = (1e-11 if prec == "fp64" else 2e-6) + 10 * fit_tol(eps, prec)
    assert np.linalg.norm(phi.double().cpu().numpy() - rphi) / np.linalg.norm(far) < tol_phi
    rF = direct.forces(q, rg)
    tol_F = (1e-10 if prec == "fp64" else 2e-5) + 100 * fit_tol(eps, prec)
    assert np.linalg.norm(F.double().cpu().numpy() - rF) / np.linalg.norm(rF) < tol_F
    ref, _ = direct.longrange_r2(x, q, L, c.rc, c.cs, grad=False)
    assert np.linalg.norm(phi.double().cpu().numpy() - ref) / np.linalg.norm(far) < eps
