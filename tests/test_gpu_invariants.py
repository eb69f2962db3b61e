"""Invariants of the long-range sum on the GPU, independent of the oracle:

* translation invariance of phi (Sec. 3.1; within eps: the grid breaks it at the eps level);
* sum of the forces ~ 0 (momentum conservation, within eps of sum |F|);
* scale covariance: the system scaled by s with r_c scaled gives phi / s and F / s^2 (Sec. 6.1,
  eq. phinondim) to rounding, since m, P and c_s are unchanged;
* linearity in the charges: phi(a q) = a phi(q), E(a q) = a^2 E(q);
* permutation equivariance, and a batch of identical systems giving identical results.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pw = pytest.importorskip("paper_2602_16591_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def run(c, x, q, prec="fp64", **kw):
    dt = torch.float32 if prec == "fp32" else torch.float64
    plan = pw.Plan(c, prec, n_max=len(q))
    phi, F, E = plan.compute(torch.as_tensor(x, dtype=dt, device=dev()), torch.as_tensor(q, dtype=dt, device=dev()),
                             **kw)
    return phi.double().cpu().numpy(), F.double().cpu().numpy(), float(E.cpu()[0])


@pytest.mark.parametrize("eps", [1e-6, 1e-10])
def test_translation_invariance_and_momentum(eps):
    x, q, L = W.paper_default(2000, seed=91)
    c = pw.choose_params(eps, L, rc=0.12)
    phi, F, E = run(c, x, q)
    shift = np.random.Generator(np.random.PCG64(92)).uniform(0, L, 3)
    phi2, F2, E2 = run(c, np.mod(x + shift, L), q)
    far = phi + (2.0 / (c.rc * c.lambda0_s)) * q     # phi_far (the self term removed)
    assert np.linalg.norm(phi2 - phi) <= 3 * eps * np.linalg.norm(far)
    assert np.linalg.norm(F2 - F) <= 30 * eps * np.linalg.norm(F)
    assert np.linalg.norm(F.sum(axis=0)) <= 10 * eps * np.abs(F).sum()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_scale_covariance(prec):
    x, q, L = W.uniform_pm1(1500, seed=93)
    s = 2.0
    c1 = pw.choose_params(1e-6, L, rc=0.1)
    c2 = pw.choose_params(1e-6, s * L, rc=0.1 * s)
    assert (c1.m, c1.P) == (c2.m, c2.P) and abs(c1.cs - c2.cs) < 1e-12
    phi1, F1, E1 = run(c1, x, q, prec)
    phi2, F2, E2 = run(c2, s * x, q, prec)
    tol = 1e-12 if prec == "fp64" else 3e-6
    assert np.linalg.norm(phi2 * s - phi1) <= tol * np.linalg.norm(phi1)
    assert np.linalg.norm(F2 * s * s - F1) <= tol * np.linalg.norm(F1)
    assert abs(E2 * s - E1) <= tol * abs(E1)


def test_linearity_in_charges():
    x, q, L = W.paper_default(1200, seed=94)
    c = pw.choose_params(1e-10, L, rc=0.15)
    phi, F, E = run(c, x, q)
    phi3, F3, E3 = run(c, x, -3.0 * q)
    assert np.max(np.abs(phi3 + 3.0 * phi)) <= 1e-12 * np.max(np.abs(phi))
    # forces are -q grad phi: quadratic in q
    assert np.max(np.abs(F3 - 9.0 * F)) <= 1e-12 * np.max(np.abs(F))
    assert abs(E3 - 9.0 * E) <= 1e-12 * abs(E)


def test_permutation_equivariance_and_identical_batch():
    x, q, L = W.uniform_pm1(1800, seed=95)
    c = pw.choose_params(1e-8, L, rc=0.12)
    phi, F, E = run(c, x, q)
    perm = np.random.Generator(np.random.PCG64(96)).permutation(len(q))
    phip, Fp, Ep = run(c, x[perm], q[perm])
    assert np.max(np.abs(phip - phi[perm])) <= 1e-12 * np.max(np.abs(phi))
    assert np.max(np.abs(Fp - F[perm])) <= 1e-11 * np.max(np.abs(F))
    assert abs(Ep - E) <= 1e-12 * abs(E)
    plan = pw.BatchPlan([c] * 3, [len(q)] * 3, "fp64")
    X = torch.as_tensor(np.concatenate([x] * 3), dtype=torch.float64, device=dev())
    Q = torch.as_tensor(np.concatenate([q] * 3), dtype=torch.float64, device=dev())
    bphi, bF, bE = plan.compute(X, Q)
    for k, part in enumerate(plan.split(bphi.cpu().numpy())):
        assert np.max(np.abs(part - phi)) <= 1e-12 * np.max(np.abs(phi)), k
    assert np.max(np.abs(bE.cpu().numpy() - E)) <= 1e-12 * abs(E)
