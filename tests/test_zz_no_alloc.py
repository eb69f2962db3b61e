"""pswfe_compute_noalloc (the entry point for callers that cannot allocate device memory) through
the C-ABI, against pswfe_compute on a plan with the same parameters: two calls in a row, the
second with a smaller input, then the first configuration again, in both precisions; and the
size limit of its device array, which is checked before any device work."""
import ctypes

import numpy as np
import pytest

import elementwise as EW
import workloads as W
from oracle import direct, fast, params as oparams

torch = pytest.importorskip("torch")
pw = pytest.importorskip("paper_2602_16591_amd")


def _noalloc(c, prec, X, Q):
    """One pswfe_compute_noalloc call through ctypes; returns (phi, force, energy)."""
    n = int(X.shape[0])
    phi = torch.full((n,), float("nan"), dtype=X.dtype, device=X.device)
    F = torch.full((n, 3), float("nan"), dtype=X.dtype, device=X.device)
    E = torch.full((1,), float("nan"), dtype=torch.float64, device=X.device)
    st = pw._lib().pswfe_compute_noalloc(ctypes.byref(c), pw.PRECISIONS[prec], n, X.data_ptr(),
                                         Q.data_ptr(), phi.data_ptr(), F.data_ptr(), E.data_ptr(),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == pw.OK, pw._lib().pswfe_status_str(st)
    return phi, F, E


def _same(name, a, b, prec, n):
    """The two entry points run the same kernels; only the order of the float64 atomic sums in the
    grid differs. Per particle: 6x the batched-vs-sequential relative bound (1e-6 float32, 1e-12
    float64) times the RMS, plus a few units of roundoff of the value itself."""
    u = 1.2e-16 if prec == "fp64" else 6e-8
    g = 1e-12 if prec == "fp64" else (2e-6 if prec == "fp32_arith" else 1e-6)
    a = a.double().cpu().numpy().reshape(n, -1)
    b = b.double().cpu().numpy().reshape(n, -1)
    assert np.isfinite(a).all()
    rms = float(np.sqrt(np.mean(np.sum(b ** 2, axis=1))))
    tol = 6 * g * rms + 4 * u * np.abs(b) + 1e-300
    r = float(np.max(np.abs(a - b) / tol))
    EW.RATIOS.append((name, r))
    assert r <= 1.0, (name, r)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_plan_on_two_calls(prec):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    dev = torch.device("cuda:0")
    dt = torch.float32 if prec == "fp32" else torch.float64
    eps = 1e-6
    first = W.uniform_pm1(6000, seed=71, L=1.2)
    second = W.paper_default(2500, seed=72, L=0.9)       # smaller input, other box and grid
    runs = []
    for (x, q, L), m in ((first, 32), (second, 24), (first, 32)):
        c = pw.choose_params(eps, L, m=m)
        X = torch.as_tensor(x, dtype=dt, device=dev)
        Q = torch.as_tensor(q, dtype=dt, device=dev)
        phi, F, E = _noalloc(c, prec, X, Q)
        plan = pw.Plan(c, prec, n_max=len(q))
        rp, rF, rE = plan.compute(X, Q)
        torch.cuda.synchronize()
        n = len(q)
        tag = f"noalloc-{prec}-n{n}-call{len(runs)}"
        _same(tag + "-phi", phi, rp, prec, n)
        _same(tag + "-force", F, rF, prec, n)
        assert abs(float(E[0]) - float(rE[0])) <= (1e-6 if prec == "fp32" else 1e-12) * abs(float(rE[0]))
        # and the parity bar of every compute path: the float64 oracle, particle by particle
        xr = x.astype(np.float32).astype(np.float64) if prec == "fp32" else x
        qr = q.astype(np.float32).astype(np.float64) if prec == "fp32" else q
        o = oparams.choose(eps, L, m=m)
        rphi, rg, grids = fast.fast_longrange(xr, qr, o, return_grids=True)
        far = rphi - direct.self_term(qr, o.rc, o.cs)
        EW.check(tag, phi.cpu().numpy(), F.cpu().numpy(), qr, rphi, rg, far, grids["b"], np.mod(xr, o.L), o,
                 pw.host_tables(c, prec)["coef"], eps, prec)
        plan.close()
        runs.append(n)
    assert runs == [6000, 2500, 6000]


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["two_level_binning", "spread_by_columns"])
def test_noalloc_matches_plan_in_the_forms_of_large_systems(case):
    """The forms large systems take, through the entry point that allocates nothing: 300,000
    particles on 64^3 (two-level binning, float32 arithmetic) and float64 on 128^3 (4,096 tiles:
    spreading by columns of tiles); then the first configuration of the other test again."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    dev = torch.device("cuda:0")
    if case == "two_level_binning":
        prec, (x, q, L), m = "fp32_arith", W.uniform_pm1(300_000, seed=73, L=2.0), 64
    else:
        prec, (x, q, L), m = "fp64", W.uniform_pm1(100_000, seed=74, L=1.0), 128
    dt = torch.float64 if prec == "fp64" else torch.float32
    c = pw.choose_params(1e-6, L, m=m)
    X = torch.as_tensor(x, dtype=dt, device=dev)
    Q = torch.as_tensor(q, dtype=dt, device=dev)
    phi, F, E = _noalloc(c, prec, X, Q)
    plan = pw.Plan(c, prec, n_max=len(q))
    rp, rF, rE = plan.compute(X, Q)
    torch.cuda.synchronize()
    n = len(q)
    _same(f"noalloc-{case}-phi", phi, rp, prec, n)
    _same(f"noalloc-{case}-force", F, rF, prec, n)
    scale = 0.5 * float(torch.sum(torch.abs(Q.double() * rp.double())))
    assert abs(float(E[0]) - float(rE[0])) <= (1e-12 if prec == "fp64" else 2e-6) * scale
    plan.close()
    # a small configuration afterwards on the same array
    x2, q2, L2 = W.uniform_pm1(6000, seed=71, L=1.2)
    c2 = pw.choose_params(1e-6, L2, m=32)
    X2 = torch.as_tensor(x2, dtype=dt, device=dev)
    Q2 = torch.as_tensor(q2, dtype=dt, device=dev)
    phi2, F2, _ = _noalloc(c2, prec, X2, Q2)
    plan2 = pw.Plan(c2, prec, n_max=len(q2))
    rp2, rF2, _ = plan2.compute(X2, Q2)
    torch.cuda.synchronize()
    _same(f"noalloc-{case}-after-phi", phi2, rp2, prec, len(q2))
    plan2.close()


def test_noalloc_refuses_configurations_beyond_its_array():
    """216^3 float64 with 1e6 particles needs about 220 MiB: refused with PSWFE_E_CAPACITY before
    any device work (so this runs without a GPU)."""
    c = pw.choose_params(1e-10, 1.0, rc=0.034370)
    assert c.m >= 216
    st = pw._lib().pswfe_compute_noalloc(ctypes.byref(c), pw.FP64, 1_000_000, None, None, None, None, None, None)
    assert st == pw.E_ARG   # pos and q are required for n > 0
    dummy = ctypes.c_void_p(16)
    st = pw._lib().pswfe_compute_noalloc(ctypes.byref(c), pw.FP64, 1_000_000, dummy, dummy, None, None, None, None)
    assert st == pw.E_CAPACITY
    assert pw._lib().pswfe_compute_noalloc(None, pw.FP64, 0, None, None, None, None, None, None) == pw.E_ARG
    assert pw._lib().pswfe_compute_noalloc(ctypes.byref(c), 7, 0, None, None, None, None, None, None) == pw.E_PREC
