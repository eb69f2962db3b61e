"""GPU parity of the real-space residual (Sec. 3.1.1) and of the full Ewald sum it completes.

* phi_local, its forces and energy against the oracle's pair sum (oracle/direct.local_direct),
  with cell lists (nc >= 3) and with every pair (tiny systems), single and batched plans;
* the full sum phi_far + phi_local + phi_self against the classical Gaussian Ewald sum and the
  oracle's split-independent total, the NaCl Madelung constant, and forces against central
  differences of the total energy.
"""
import math

import numpy as np
import pytest

import workloads as W
from conftest import read_table
from oracle import direct, params as oparams

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pw = pytest.importorskip("paper_2602_16591_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def dt(prec):
    return torch.float32 if prec == "fp32" else torch.float64


def rounded(a, prec):
    return np.asarray(a, dtype=np.float32 if prec == "fp32" else np.float64).astype(np.float64)


def tdev(a, prec):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt(prec), device=dev())


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


LOCAL_CASES = [
    # (name, generator, eps, params kwargs): cell counts floor(L / r_c) of 7, 3 and 2 (all pairs)
    ("uniform_cells7", lambda: W.uniform_pm1(1500, seed=41), 1e-6, dict(m=32)),
    ("paper_cells3", lambda: W.paper_default(300, seed=42, L=1.2), 1e-6, dict(m=16)),
    ("tiny_all_pairs", lambda: W.paper_default(40, seed=43, L=0.9), 1e-6, dict(m=12)),
    ("clustered_fp64_eps", lambda: W.clustered(1200, seed=44, L=1.0), 1e-10, dict(m=40)),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", LOCAL_CASES, ids=[c[0] for c in LOCAL_CASES])
def test_local_matches_oracle(case, prec):
    _, gen, eps, kw = case
    if prec == "fp32" and eps < 1e-6:
        pytest.skip("fp32 path is for eps >= 1e-6")
    x, q, L = gen()
    x, q = rounded(x, prec), rounded(q, prec)
    c = pw.choose_params(eps, L, **kw)
    o = oparams.choose(eps, L, **kw)
    assert o.rc < L / 2
    plan = pw.Plan(c, prec, n_max=len(q))
    phi, F, E = plan.local(tdev(x, prec), tdev(q, prec))
    rphi, rg = direct.local_direct(x, q, L, o.rc, o.cs)
    rF = direct.forces(q, rg)
    tol = 1e-12 if prec == "fp64" else 2e-7
    assert rel_l2(phi.cpu().numpy(), rphi) < tol
    assert rel_l2(F.cpu().numpy(), rF) < 10 * tol
    Eref = 0.5 * float(np.dot(q, rphi))
    assert abs(float(E.cpu()[0]) - Eref) <= tol * 0.5 * float(np.abs(q) @ np.abs(rphi))
    # grad mode gives grad phi_local
    _, G, _ = plan.local(tdev(x, prec), tdev(q, prec), grad=True)
    assert rel_l2(G.cpu().numpy(), rg) < 10 * tol


@pytest.mark.parametrize("threads", ["128", "256", "default"])
def test_local_workgroup_sizes_match_oracle(threads, monkeypatch):
    """Every residual workgroup size (16, 32 or 64 targets per pass; cells of ~32 particles take
    one to two passes) gives the oracle's pair sum."""
    if threads != "default":
        monkeypatch.setenv("PSWFE_LOCAL_THREADS", threads)
    x, q, L = W.uniform_pm1(4000, seed=45)
    c = pw.choose_params(1e-6, L, m=24)
    o = oparams.choose(1e-6, L, m=24)
    plan = pw.Plan(c, "fp64", n_max=len(q))
    phi, F, E = plan.local(tdev(x, "fp64"), tdev(q, "fp64"))
    rphi, rg = direct.local_direct(x, q, L, o.rc, o.cs)
    assert rel_l2(phi.cpu().numpy(), rphi) < 1e-12
    assert rel_l2(F.cpu().numpy(), direct.forces(q, rg)) < 1e-11
    assert abs(float(E.cpu()[0]) - 0.5 * float(np.dot(q, rphi))) <= 1e-12 * 0.5 * float(np.abs(q) @ np.abs(rphi))


def test_total_matches_gaussian_ewald():
    """phi_far + phi_local + phi_self at eps = 1e-10 against the classical Gaussian split
    converged to ~1e-14 (Example 1): the total does not depend on the split."""
    x, q, L = W.paper_default(80, seed=45, L=1.3)
    c = pw.choose_params(1e-10, L, m=24)
    plan = pw.Plan(c, "fp64", n_max=len(q))
    phi, F, E = plan.compute(tdev(x, "fp64"), tdev(q, "fp64"), total=True)
    pg, gg = direct.gauss_ewald(x, q, L)
    assert rel_l2(phi.cpu().numpy(), pg) < 2e-9
    assert rel_l2(F.cpu().numpy(), direct.forces(q, gg)) < 2e-8
    assert abs(float(E.cpu()[0]) - 0.5 * float(q @ pg)) < 2e-9 * 0.5 * float(np.abs(q) @ np.abs(pg))


@pytest.mark.parametrize("a", [1.0, 2.5])
def test_madelung_constant(a):
    """Rock-salt cell on the GPU (full Ewald sum, eps = 1e-10): phi_i = -q_i M / (a/2) with the
    textbook Madelung constant; every force vanishes by symmetry."""
    M = float(read_table("madelung_nacl.txt")[0][0])
    x, q, L = W.nacl_cell(a)
    c = pw.choose_params(1e-10, L, m=20)   # r_c = 0.37 L: every pair (fewer than 3 cells)
    plan = pw.Plan(c, "fp64", n_max=len(q))
    phi, F, E = plan.compute(tdev(x, "fp64"), tdev(q, "fp64"), total=True)
    np.testing.assert_allclose(phi.cpu().numpy(), -q * M / (a / 2), rtol=1e-9, atol=0)
    assert abs(float(E.cpu()[0]) + 4.0 * M / (a / 2)) < 1e-9 * 4 * M / (a / 2)
    assert float(F.abs().max()) < 1e-8 * M / (a / 2) ** 2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_total_forces_are_energy_gradients(prec):
    """F_total = -dE_total/dx by central differences of the float64 total energy, away from
    stencil shifts, and dE/dq = phi_total through autograd."""
    from paper_2602_16591_amd import autograd as ag
    x, q, L = W.uniform_pm1(600, seed=46, L=1.1)
    x = x.astype(np.float32).astype(np.float64)
    c = pw.choose_params(1e-6, L, m=24)
    o = oparams.choose(1e-6, L, m=24)
    plan = pw.Plan(c, prec, n_max=len(q))
    X = torch.tensor(x, dtype=dt(prec), device=dev(), requires_grad=True)
    Q = torch.tensor(q, dtype=dt(prec), device=dev(), requires_grad=True)
    E, phi = ag.energy_and_potential(X, Q, plan, total=True)
    E.sum().backward()
    assert torch.equal(Q.grad, phi.detach())
    _, F, _ = plan.compute(X.detach(), Q.detach(), total=True)
    assert torch.allclose(X.grad, -F, rtol=1e-6, atol=1e-6 * float(F.abs().max()))
    p64 = pw.Plan(c, "fp64", n_max=len(q))
    X64, Q64 = tdev(x, "fp64"), tdev(q, "fp64")
    hfd = 1e-6 * L
    rng = np.random.Generator(np.random.PCG64(47))
    Fn = F.double().cpu().numpy()
    errs = []
    for i in rng.choice(len(q), 60, replace=False):
        d = int(rng.integers(0, 3))
        t = x[i, d] / o.h - o.P / 2.0
        if min(t - math.floor(t), math.ceil(t) - t) < 4 * hfd / o.h:
            continue
        Ep = []
        for sgn in (1, -1):
            Xp = X64.clone()
            Xp[i, d] += sgn * hfd
            Ep.append(float(p64.compute(Xp, Q64, phi=False, force=False, total=True)[2].cpu()[0]))
        errs.append(-(Ep[0] - Ep[1]) / (2 * hfd) - Fn[i, d])
    assert len(errs) > 40
    tol = 1e-6 if prec == "fp64" else 3e-5
    assert np.sqrt(np.mean(np.square(errs))) < tol * np.sqrt(np.mean(Fn ** 2))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_total_matches_single_and_oracle(prec):
    systems = [W.uniform_pm1(500, seed=48, L=1.0), W.paper_default(40, seed=49, L=0.9),
               W.clustered(700, seed=50, L=1.3)]
    grids = [24, 12, 30]
    params = [pw.choose_params(1e-6, L, m=m) for (_, _, L), m in zip(systems, grids)]
    counts = [len(q) for _, q, _ in systems]
    xs = [rounded(s[0], prec) for s in systems]
    qs = [rounded(s[1], prec) for s in systems]
    plan = pw.BatchPlan(params, counts, prec)
    X, Q = tdev(np.concatenate(xs), prec), tdev(np.concatenate(qs), prec)
    phi, F, E = plan.compute(X, Q, total=True)
    lphi, lF, lE = plan.split(phi.cpu().numpy()), plan.split(F.cpu().numpy()), E.cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-6
    for k in range(3):
        single = pw.Plan(params[k], prec, n_max=counts[k])
        sp, sF, sE = single.compute(tdev(xs[k], prec), tdev(qs[k], prec), total=True)
        assert rel_l2(lphi[k], sp.cpu().numpy()) < tol
        assert rel_l2(lF[k], sF.cpu().numpy()) < tol
        assert abs(lE[k] - float(sE.cpu()[0])) <= tol * abs(lE[k])
        # the residual part alone against the oracle
        L = systems[k][2]
        o = oparams.choose(1e-6, L, m=grids[k])
        far, _, _ = single.compute(tdev(xs[k], prec), tdev(qs[k], prec))
        loc = sp.double().cpu().numpy() - far.double().cpu().numpy()
        rphi, _ = direct.local_direct(xs[k], qs[k], L, o.rc, o.cs, grad=False)
        assert rel_l2(loc, rphi) < (1e-11 if prec == "fp64" else 2e-5)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_water_box_total_potential(prec):
    """The water box (n = 30,000, eps = 1e-6 absolute RMS, 64^3): the full Ewald potential against
    the oracle's split-independent total on 96 sampled sites."""
    x, q, L = W.config("water_n30000")
    x, q = rounded(x, prec), rounded(q, prec)
    eps = 1e-6
    qn = float(np.linalg.norm(q))
    c = pw.choose_params(eps, L, m=64, q_l2=qn, tol_mode="abs")
    plan = pw.Plan(c, prec, n_max=len(q))
    phi, F, E = plan.compute(tdev(x, prec), tdev(q, prec), total=True)
    idx = np.sort(np.random.Generator(np.random.PCG64(51)).choice(len(q), 96, replace=False))
    ref, gref = direct.total_potential(x, q, L, target_idx=idx, rc_o=0.3 * L, cs_o=30.0)
    err = phi.double().cpu().numpy()[idx] - ref
    assert np.sqrt(np.mean(err ** 2)) < 1.5 * eps


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_overlapped_residual_matches_sequential(prec, monkeypatch):
    """The residual computed on the plan's side stream, alongside the long-range part, and added
    by the interpolation in float64 gives the results of computing it afterwards on the caller's
    stream (one rounding instead of two; energies within rounding)."""
    x, q, L = W.uniform_pm1(3000, seed=47)
    x, q = rounded(x, prec), rounded(q, prec)
    c = pw.choose_params(1e-6, L, m=32)
    out = {}
    for overlap in ("1", "0"):
        monkeypatch.setenv("PSWFE_LOCAL_OVERLAP", overlap)
        plan = pw.Plan(c, prec, n_max=len(q))
        phi, F, E = plan.compute(tdev(x, prec), tdev(q, prec), total=True)
        _, G, _ = plan.compute(tdev(x, prec), tdev(q, prec), total=True, grad=True)
        out[overlap] = [a.double().cpu().numpy() for a in (phi, F, G, E)]
        plan.close()
    tol = 1e-13 if prec == "fp64" else 2e-7
    for a, b in zip(out["1"][:3], out["0"][:3]):
        assert rel_l2(a, b) < tol
    assert abs(out["1"][3][0] - out["0"][3][0]) <= tol * abs(out["0"][3][0])
    # batch plans take the same path
    monkeypatch.setenv("PSWFE_LOCAL_OVERLAP", "1")
    bplan = pw.BatchPlan([c, c], [len(q), len(q)], prec)
    X2 = tdev(np.concatenate([x, x]), prec)
    Q2 = tdev(np.concatenate([q, -q]), prec)
    bphi, bF, bE = bplan.compute(X2, Q2, total=True)
    bphi = bphi.double().cpu().numpy()
    assert rel_l2(bphi[:len(q)], out["0"][0]) < 10 * tol
    assert rel_l2(bphi[len(q):], -out["0"][0]) < 10 * tol
    assert np.allclose(bE.cpu().numpy(), out["0"][3][0], rtol=10 * tol, atol=0)


def test_graph_replay_of_the_total_sum():
    """A captured graph of the full Ewald sum (the residual forked to the side stream and joined
    back inside the capture) replays to the eager results, with eager work between replays and
    new inputs."""
    prec = "fp32"
    x, q, L = W.uniform_pm1(4000, seed=48)
    c = pw.choose_params(1e-6, L, m=32)
    plan = pw.Plan(c, prec, n_max=len(q))
    X, Q = tdev(x, prec), tdev(q, prec)
    e_phi, e_F, e_E = plan.compute(X, Q, total=True)
    torch.cuda.synchronize()
    runner = plan.graph(X, Q, total=True)
    other = pw.Plan(c, prec, n_max=len(q))
    for _ in range(4):
        phi, F, E = runner()
        torch.cuda.synchronize()
        assert torch.allclose(phi, e_phi, rtol=0, atol=1e-6 * float(e_phi.abs().max()))
        assert torch.allclose(F, e_F, rtol=0, atol=1e-6 * float(e_F.abs().max()))
        assert torch.allclose(E, e_E, rtol=1e-6, atol=1e-12)
        other.compute(X, Q, total=True)
        _ = (X * 2).sum()
        torch.cuda.synchronize()
    phi2, F2, E2 = runner(q=-Q)
    torch.cuda.synchronize()
    assert torch.allclose(phi2, -e_phi, rtol=0, atol=1e-6 * float(e_phi.abs().max()))
    assert torch.allclose(E2, e_E, rtol=1e-6, atol=1e-12)
