"""GPU parity of batched plans (many independent systems per launch) through the C-ABI.

* each system of a batch against Alg. 2 in float64 (oracle/fast.py) at its own parameters;
* batched against sequential single-system plans with the same parameters and tiles (the same
  arithmetic; only the order of the float64 atomic additions into the grid may differ, which
  moves a float32 result by a few units in the last place at most);
* a captured HIP graph against eager calls, over several replays with eager work between;
* the tile autotuner's plan against the default plan;
* the full ensemble workload: 256 systems of uneven sizes, every system against its
  sequential plan and 16 seeded systems against the oracle.
"""
import numpy as np
import pytest

import elementwise as EW
import workloads as W
from oracle import direct, fast, params as oparams

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pw = pytest.importorskip("paper_2602_16591_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def dt(prec):
    return torch.float64 if prec == "fp64" else torch.float32


def rounded(a, prec):
    return np.asarray(a, dtype=np.float64 if prec == "fp64" else np.float32).astype(np.float64)


def fit_tol(eps, prec):
    return max(0.01 * eps, 1e-15 if prec == "fp64" else 5e-9)


def pack(systems, prec):
    x = np.concatenate([s[0] for s in systems]) if systems else np.zeros((0, 3))
    q = np.concatenate([s[1] for s in systems]) if systems else np.zeros(0)
    d = dev()
    return (torch.as_tensor(rounded(x, prec), dtype=dt(prec), device=d),
            torch.as_tensor(rounded(q, prec), dtype=dt(prec), device=d))


def check_vs_oracle(x, q, o, phi, F, E, eps, prec, c=None, name="batch"):
    """The compute parity bar of the single-system tests, for one system: norms, and with the
    library parameters c the per-particle bounds of tests/elementwise.py."""
    if len(q) == 0:
        assert E == 0.0
        return
    rphi, rg, grids = fast.fast_longrange(x, q, o, return_grids=True)
    rF = direct.forces(q, rg)
    far = rphi - direct.self_term(q, o.rc, o.cs)
    if c is not None and len(q) > 1:
        EW.check(name, phi, F, q, rphi, rg, far, grids["b"], np.mod(x, o.L), o, pw.host_tables(c, prec)["coef"],
                 eps, prec)
    tol_phi = (1e-11 if prec == "fp64" else 2e-6) + 10 * fit_tol(eps, prec)
    tol_F = (1e-10 if prec == "fp64" else 2e-5) + 100 * fit_tol(eps, prec)
    scale = max(np.linalg.norm(far), 1e-300)
    assert np.linalg.norm(phi - rphi) / scale < tol_phi
    if len(q) > 1:   # a lone charge feels no net force from its own images: nothing relative to check
        assert np.linalg.norm(F - rF) / np.linalg.norm(rF) < tol_F
    Eref = 0.5 * float(np.dot(q, rphi))
    assert abs(E - Eref) <= tol_phi * 0.5 * np.abs(q) @ np.abs(far) + 1e-12 * abs(Eref) + 1e-300


# Systems of a small mixed batch: (generator, eps, params kwargs). Different eps give different
# P (odd and even), different L and n give different m; one system is empty, one has a single
# charge (not neutral: the k = 0 mode is dropped all the same).
MIXED = [
    (lambda: W.uniform_pm1(300, seed=11, L=1.0), 1e-6, dict(m=24)),
    (lambda: W.uniform_pm1(0, seed=12, L=0.7), 1e-6, dict(m=16)),
    (lambda: W.paper_default(500, seed=13, L=1.6), 1e-4, dict(m=20)),
    (lambda: (np.array([[0.27, 0.61, 0.05]]), np.array([1.0]), 0.9), 1e-6, dict(m=16)),
    (lambda: W.uniform_pm1(800, seed=15, L=1.2), 1e-8, dict(m=36)),
    (lambda: W.clustered(600, seed=16, L=0.8), 1e-6, dict(m=30)),
]


def mixed_systems(prec):
    out = []
    for gen, eps, kw in MIXED:
        if prec != "fp64" and eps < 1e-6:
            eps = 1e-6
        x, q, L = gen()
        x, q = rounded(x, prec), rounded(q, prec)
        c = pw.choose_params(eps, L, **kw)
        o = oparams.choose(eps, L, **kw)
        assert (c.m, c.P) == (o.m, o.P)
        out.append((x, q, L, eps, c, o))
    return out


@pytest.mark.parametrize("levels", ["1", "2"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_arith"])
def test_mixed_batch_matches_oracle_and_sequential(prec, levels, monkeypatch):
    monkeypatch.setenv("PSWFE_BIN_LEVELS", levels)   # one-level or two-level binning of the batch
    systems = mixed_systems(prec)
    assert len({s[4].P for s in systems}) >= 2           # several P groups in one plan
    pos, q = pack([(s[0], s[1]) for s in systems], prec)
    plan = pw.BatchPlan([s[4] for s in systems], [len(s[1]) for s in systems], prec)
    assert plan.nsys == len(systems) and plan.n_total == pos.shape[0]
    for k, s in enumerate(systems):
        p, off, cnt, tile = plan.system(k)
        assert (p.m, p.P, cnt) == (s[4].m, s[4].P, len(s[1]))
        assert off == sum(len(t[1]) for t in systems[:k])
    phi, F, E = plan.compute(pos, q)
    E = E.cpu().numpy()
    phis, Fs = plan.split(phi.cpu().numpy()), plan.split(F.cpu().numpy())
    for k, (x, qq, L, eps, c, o) in enumerate(systems):
        check_vs_oracle(x, qq, o, phis[k], Fs[k], float(E[k]), eps, prec, c=c, name=f"mixed-batch-{prec}-bin{levels}-sys{k}")
    # sequential single-system plans with the same tiles
    tol = 1e-12 if prec == "fp64" else 1e-6
    for k, (x, qq, L, eps, c, o) in enumerate(systems):
        single = pw.Plan(c, prec, n_max=len(qq), tile=plan.tiles[k])
        assert single.tile == plan.tiles[k]
        sp, sF, sE = single.compute(*pack([(x, qq)], prec))
        if len(qq) == 0:
            assert float(sE.cpu()[0]) == 0.0 == float(E[k])
            continue
        sp, sF = sp.cpu().numpy(), sF.cpu().numpy()
        assert np.linalg.norm(phis[k] - sp) <= tol * np.linalg.norm(sp) + 1e-30
        assert np.linalg.norm(Fs[k] - sF) <= tol * np.linalg.norm(sF) + 1e-30
        assert abs(float(E[k]) - float(sE.cpu()[0])) <= tol * 0.5 * float(np.abs(qq) @ np.abs(sp)) + 1e-30
        single.close()
    # grad mode returns grad phi_far: force = -q grad phi (a second call: the float64 atomic
    # additions may round in another order)
    _, G, _ = plan.compute(pos, q, grad=True)
    assert float(torch.linalg.norm(F + q[:, None] * G)) <= tol * float(torch.linalg.norm(F))


def test_graph_replay_matches_eager():
    prec = "fp32"
    systems = mixed_systems(prec)
    pos, q = pack([(s[0], s[1]) for s in systems], prec)
    plan = pw.BatchPlan([s[4] for s in systems], [len(s[1]) for s in systems], prec)
    e_phi, e_F, e_E = plan.compute(pos, q)
    torch.cuda.synchronize()
    runner = plan.graph(pos, q)
    other = pw.Plan(systems[0][4], prec, n_max=len(systems[0][1]))
    ox, oq = pack([(systems[0][0], systems[0][1])], prec)
    for rep in range(4):
        phi, F, E = runner()
        torch.cuda.synchronize()
        assert torch.allclose(phi, e_phi, rtol=0, atol=1e-6 * float(e_phi.abs().max()))
        assert torch.allclose(F, e_F, rtol=0, atol=1e-6 * float(e_F.abs().max()))
        assert torch.allclose(E, e_E, rtol=1e-6, atol=1e-12)
        # eager work of the program between replays: other plans, torch ops, a sync
        other.compute(ox, oq)
        _ = (pos * 2).sum()
        torch.cuda.synchronize()
    # new inputs: charges flipped -> potentials, forces flip; energies stay
    phi2, F2, E2 = runner(q=-q)
    torch.cuda.synchronize()
    assert torch.allclose(phi2, -e_phi, rtol=0, atol=1e-6 * float(e_phi.abs().max()))
    assert torch.allclose(E2, e_E, rtol=1e-6, atol=1e-12)
    # and the single-system plan captured the same way
    srun = other.graph(ox, oq)
    s_phi, _, _ = other.compute(ox, oq)
    for _ in range(3):
        g_phi, _, _ = srun()
        torch.cuda.synchronize()
        assert torch.allclose(g_phi, s_phi, rtol=0, atol=1e-6 * float(s_phi.abs().max()))


def test_autotuner_picks_a_measured_plan():
    from paper_2602_16591_amd.autotune import autotune_batch, autotune_plan
    prec = "fp32"
    systems = mixed_systems(prec)
    params = [s[4] for s in systems]
    counts = [len(s[1]) for s in systems]
    pos, q = pack([(s[0], s[1]) for s in systems], prec)
    cache = {}
    plan, tiles, report = autotune_batch(params, counts, pos, q, prec, targets=(None, 16, 256), reps=3, cache=cache)
    assert report and plan.tiles == tiles and min(r[2] for r in report) == cache[next(iter(cache))]["ms"]
    ref = pw.BatchPlan(params, counts, prec)
    a, b = plan.compute(pos, q)[0], ref.compute(pos, q)[0]
    assert torch.allclose(a, b, rtol=0, atol=2e-6 * float(b.abs().max()))
    plan2, tiles2, report2 = autotune_batch(params, counts, pos, q, prec, cache=cache)   # cached
    assert tiles2 == tiles and report2 == []
    x, qq = systems[4][0], systems[4][1]
    sx, sq = pack([(x, qq)], prec)
    splan, t, rep = autotune_plan(systems[4][4], sx, sq, prec, tiles=(4, 6, 8), reps=3)
    assert splan.tile == t and len(rep) >= 2


def test_batch_rejects_single_entry_points_and_wrong_shapes():
    prec = "fp64"
    systems = mixed_systems(prec)[:3]
    pos, q = pack([(s[0], s[1]) for s in systems], prec)
    plan = pw.BatchPlan([s[4] for s in systems], [len(s[1]) for s in systems], prec)
    lib = pw._lib()
    assert lib.pswfe_compute(plan._h, 1, pos.data_ptr(), q.data_ptr(), None, None, None, None) == pw.E_ARG
    single = pw.Plan(systems[0][4], prec, n_max=10)
    assert lib.pswfe_batch_compute(single._h, pos.data_ptr(), q.data_ptr(), None, None, None, None) == pw.E_ARG
    with pytest.raises(ValueError):
        plan.compute(pos[:-1], q[:-1])


def _ensemble(prec):
    ens = W.ensemble()
    params = [pw.choose_params(1e-6, L, n=len(q)) for x, q, L in ens]
    return ens, params


@pytest.mark.parametrize("prec", ["fp32", "fp32_arith"])
def test_full_ensemble_batched_vs_sequential_and_oracle(prec):
    """256 systems, n log-uniform in [500, 20000], L uniform in [0.5, 2], eps = 1e-6, float32
    storage with float64 or float32 window arithmetic."""
    ens, params = _ensemble(prec)
    counts = [len(q) for _, q, _ in ens]
    pos, q = pack([(x, qq) for x, qq, _ in ens], prec)
    plan = pw.BatchPlan(params, counts, prec)
    phi, F, E = plan.compute(pos, q)
    phis, Fs, E = plan.split(phi.cpu().numpy()), plan.split(F.cpu().numpy()), E.cpu().numpy()
    # every system against its own sequential plan (same tiles): the same arithmetic up to the
    # order of the tile sums (particles within a bucket come in any order), which float32 sums
    # feel more
    tol = 2e-6 if prec == "fp32_arith" else 1e-6
    for k, (x, qq, L) in enumerate(ens):
        single = pw.Plan(params[k], prec, n_max=len(qq), tile=plan.tiles[k])
        sp, sF, sE = single.compute(*pack([(x, qq)], prec))
        sp, sF = sp.cpu().numpy(), sF.cpu().numpy()
        assert np.linalg.norm(phis[k] - sp) <= tol * np.linalg.norm(sp), k
        assert np.linalg.norm(Fs[k] - sF) <= tol * np.linalg.norm(sF), k
        # the energy of a neutral system is a small difference of large terms: its rounding, from
        # the order in which the float32 (float32 arithmetic) or float64 tile sums are taken, is
        # relative to the sum of |q_i phi_i|, not to E
        assert abs(E[k] - float(sE.cpu()[0])) <= tol * 0.5 * float(np.abs(qq) @ np.abs(sp)), k
        single.close()
    # 16 seeded systems against the oracle
    pick = np.random.default_rng(16591).choice(len(ens), 16, replace=False)
    for k in pick:
        x, qq, L = ens[k]
        x, qq = rounded(x, prec), rounded(qq, prec)
        o = oparams.choose(1e-6, L, n=len(qq))
        assert (o.m, o.P) == (params[k].m, params[k].P)
        check_vs_oracle(x, qq, o, phis[k], Fs[k], float(E[k]), 1e-6, prec, c=params[k], name=f"ensemble-sys{k}")
