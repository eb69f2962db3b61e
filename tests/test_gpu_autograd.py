"""Differentiation through the HIP path (paper_2602_16591_amd.autograd) against finite
differences of the float64 path and against the oracle's analytic forces."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct, params as oparams

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pw = pytest.importorskip("paper_2602_16591_amd")
from paper_2602_16591_amd import autograd as ag  # noqa: E402


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def away_from_shift(x, h_fd, p):
    """True where x/h - P/2 is at least 4 finite-difference steps away from an integer, so that
    x +- h_fd keeps the same support points (a support shift changes the energy by ~eps_w)."""
    t = x / p.h - p.P / 2.0
    return np.minimum(t - np.floor(t), np.ceil(t) - t) > 4 * h_fd / p.h


def test_clustered_energy_gradients():
    """n = 1e5 clustered charges, float32 at eps = 1e-6: dE/dq = phi and dE/dx = -F exactly (same
    launch), dE/dx against central differences of the float64 energy (h = 1e-4 L) on 64 sampled
    coordinates, and against the oracle's analytic forces on 32 sampled particles."""
    x, q, L = W.config("clustered_n1e5")
    x = x.astype(np.float32).astype(np.float64)
    eps = 1e-6
    c = pw.choose_params(eps, L, n=len(q))
    o = oparams.choose(eps, L, n=len(q))
    p32 = pw.Plan(c, "fp32", n_max=len(q))
    X = torch.tensor(x, dtype=torch.float32, device=dev(), requires_grad=True)
    Q = torch.tensor(q, dtype=torch.float32, device=dev(), requires_grad=True)
    E, phi = ag.energy_and_potential(X, Q, p32)
    E.sum().backward()
    _, F, _ = p32.compute(X.detach(), Q.detach())
    assert torch.equal(Q.grad, phi.detach())
    assert torch.allclose(X.grad, -F, rtol=1e-6, atol=1e-6 * float(F.abs().max()))
    dEdx = X.grad.double().cpu().numpy()
    # finite differences of the float64 path
    p64 = pw.Plan(c, "fp64", n_max=len(q))
    X64 = torch.tensor(x, dtype=torch.float64, device=dev())
    Q64 = torch.tensor(q, dtype=torch.float64, device=dev())
    hfd = 1e-4 * L
    rng = np.random.Generator(np.random.PCG64(4))
    checked = 0
    errs, scale = [], []
    for i in rng.choice(len(q), 200, replace=False):
        d = int(rng.integers(0, 3))
        if not away_from_shift(x[i, d], hfd, o):
            continue
        Ep = []
        for sgn in (1, -1):
            Xp = X64.clone()
            Xp[i, d] += sgn * hfd
            Ep.append(float(p64.compute(Xp, Q64, phi=False, force=False)[2].cpu()[0]))
        errs.append((Ep[0] - Ep[1]) / (2 * hfd) - dEdx[i, d])
        scale.append(abs(dEdx[i, d]))
        checked += 1
        if checked == 64:
            break
    assert checked == 64
    rms_F = float(np.sqrt(np.mean(dEdx ** 2)))
    assert np.sqrt(np.mean(np.square(errs))) < 1e-4 * rms_F
    # oracle analytic forces (direct sum, route R2) on sampled particles
    idx = np.sort(rng.choice(len(q), 32, replace=False))
    ref, gref = direct.longrange_r2(x, q, L, o.rc, o.cs, target_idx=idx, rc_o=0.3 * L, cs_o=30.0)
    Fref = direct.forces(q[idx], gref)
    kmax = o.m // 2
    far = ref - direct.self_term(q[idx], o.rc, o.cs)
    bound = 3 * (2 * math.pi * kmax / L) * eps * np.sqrt(np.mean(far ** 2)) * np.sqrt(np.mean(q[idx] ** 2))
    assert np.sqrt(np.mean(np.sum((-dEdx[idx] - Fref) ** 2, axis=1))) < max(bound, 1e-5 * rms_F)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_general_loss_adjoint(prec):
    """L = sum_i w_i phi_i + 0.3 E: gradients in q and x from the adjoint (a second application
    with charges w) against central differences of the float64 path."""
    x, q, L = W.uniform_pm1(2000, seed=12, L=1.7)
    x = x.astype(np.float32).astype(np.float64)
    c = pw.choose_params(1e-6, L, m=32)
    o = oparams.choose(1e-6, L, m=32)
    dt = torch.float32 if prec == "fp32" else torch.float64
    plan = pw.Plan(c, prec, n_max=len(q))
    rng = np.random.Generator(np.random.PCG64(13))
    w = rng.standard_normal(len(q))
    X = torch.tensor(x, dtype=dt, device=dev(), requires_grad=True)
    Q = torch.tensor(q, dtype=dt, device=dev(), requires_grad=True)
    Wt = torch.tensor(w, dtype=dt, device=dev())
    E, phi = ag.energy_and_potential(X, Q, plan)
    loss = (Wt * phi).sum() + 0.3 * E.to(dt).sum()
    loss.backward()
    gx, gq = X.grad.double().cpu().numpy(), Q.grad.double().cpu().numpy()
    p64 = pw.Plan(c, "fp64", n_max=len(q))
    X64 = torch.tensor(x, dtype=torch.float64, device=dev())
    Q64 = torch.tensor(q, dtype=torch.float64, device=dev())
    W64 = torch.tensor(w, dtype=torch.float64, device=dev())

    def L_of(Xv, Qv):
        ph, _, En = p64.compute(Xv, Qv, force=False)
        return float((W64 * ph).sum().cpu()) + 0.3 * float(En.cpu()[0])

    # charges: L is quadratic in q, so the central difference is exact up to rounding
    for i in rng.choice(len(q), 8, replace=False):
        Qp, Qm = Q64.clone(), Q64.clone()
        Qp[i] += 1e-3
        Qm[i] -= 1e-3
        fd = (L_of(X64, Qp) - L_of(X64, Qm)) / 2e-3
        assert abs(fd - gq[i]) < (1e-8 if prec == "fp64" else 3e-5) * np.max(np.abs(gq))
    hfd = 1e-5 * L
    errs = []
    for i in rng.choice(len(q), 64, replace=False):
        d = int(rng.integers(0, 3))
        if not away_from_shift(x[i, d], hfd, o):
            continue
        Xp, Xm = X64.clone(), X64.clone()
        Xp[i, d] += hfd
        Xm[i, d] -= hfd
        errs.append((L_of(Xp, Q64) - L_of(Xm, Q64)) / (2 * hfd) - gx[i, d])
    assert len(errs) > 40
    tol = 1e-6 if prec == "fp64" else 3e-5
    assert np.sqrt(np.mean(np.square(errs))) < tol * np.sqrt(np.mean(gx ** 2))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_adjoint_matches_single_systems(prec):
    """A batch of three systems with L = sum_s c_s E_s + sum_i w_i phi_i: the batched adjoint
    against each system's own single-plan adjoint, and the charge gradients against central
    differences of the float64 batch (L is quadratic in q)."""
    systems = [W.uniform_pm1(400, seed=31, L=1.0), W.uniform_pm1(600, seed=32, L=1.5),
               W.paper_default(500, seed=33, L=0.8)]
    grids = [24, 30, 20]
    dt = torch.float32 if prec == "fp32" else torch.float64
    params = [pw.choose_params(1e-6, L, m=m) for (_, _, L), m in zip(systems, grids)]
    counts = [len(q) for _, q, _ in systems]
    x = np.concatenate([s[0] for s in systems]).astype(np.float32).astype(np.float64)
    q = np.concatenate([s[1] for s in systems])
    rng = np.random.Generator(np.random.PCG64(34))
    w = rng.standard_normal(len(q))
    cs = np.array([0.7, -1.3, 2.1])
    plan = pw.BatchPlan(params, counts, prec)
    X = torch.tensor(x, dtype=dt, device=dev(), requires_grad=True)
    Q = torch.tensor(q, dtype=dt, device=dev(), requires_grad=True)
    E, phi = ag.batch_energy_and_potential(X, Q, plan)
    loss = (torch.tensor(w, dtype=dt, device=dev()) * phi).sum() + (torch.tensor(cs, device=dev()) * E).sum().to(dt)
    loss.backward()
    gx, gq = X.grad.double().cpu().numpy(), Q.grad.double().cpu().numpy()
    tol = 1e-10 if prec == "fp64" else 1e-5
    for s, (o, n) in enumerate(zip(plan.offsets, plan.counts)):
        sp = pw.Plan(params[s], prec, n_max=n)
        Xs = torch.tensor(x[o:o + n], dtype=dt, device=dev(), requires_grad=True)
        Qs = torch.tensor(q[o:o + n], dtype=dt, device=dev(), requires_grad=True)
        Es, phis = ag.energy_and_potential(Xs, Qs, sp)
        ls = (torch.tensor(w[o:o + n], dtype=dt, device=dev()) * phis).sum() + cs[s] * Es.to(dt).sum()
        ls.backward()
        rx, rq = Xs.grad.double().cpu().numpy(), Qs.grad.double().cpu().numpy()
        assert np.linalg.norm(gx[o:o + n] - rx) <= tol * np.linalg.norm(rx)
        assert np.linalg.norm(gq[o:o + n] - rq) <= tol * np.linalg.norm(rq)
    p64 = pw.BatchPlan(params, counts, "fp64")
    X64 = torch.tensor(x, dtype=torch.float64, device=dev())
    W64 = torch.tensor(w, dtype=torch.float64, device=dev())
    C64 = torch.tensor(cs, dtype=torch.float64, device=dev())

    def L_of(Qv):
        ph, _, En = p64.compute(X64, Qv, force=False)
        return float((W64 * ph).sum().cpu()) + float((C64 * En).sum().cpu())

    Q64 = torch.tensor(q, dtype=torch.float64, device=dev())
    for i in [5, counts[0] + 7, counts[0] + counts[1] + 11]:
        Qp, Qm = Q64.clone(), Q64.clone()
        Qp[i] += 1e-3
        Qm[i] -= 1e-3
        fd = (L_of(Qp) - L_of(Qm)) / 2e-3
        assert abs(fd - gq[i]) < (1e-8 if prec == "fp64" else 3e-5) * np.max(np.abs(gq))
