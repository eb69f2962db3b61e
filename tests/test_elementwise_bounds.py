"""CPU checks of the per-particle parity bounds (tests/elementwise.py) that the GPU tests use:
results the bounds must accept (the oracle's own values, rounded to the working precision) and
planted mistakes they must reject (one particle's potential or one force component off, a
support shifted by a grid point). The mistakes are planted in copies of the oracle's output."""
import numpy as np
import pytest

import elementwise as EW
import workloads as W
from oracle import direct, fast, params as oparams

pw = pytest.importorskip("paper_2602_16591_amd")


def _system(prec, eps=1e-6, m=24, n=400, seed=41):
    x, q, L = W.uniform_pm1(n, seed=seed)
    dt = np.float64 if prec == "fp64" else np.float32
    x = x.astype(dt).astype(np.float64)
    q = q.astype(dt).astype(np.float64)
    c = pw.choose_params(eps, L, m=m)
    o = oparams.choose(eps, L, m=m)
    rphi, rg, grids = fast.fast_longrange(x, q, o, return_grids=True)
    far = rphi - direct.self_term(q, o.rc, o.cs)
    coef = pw.host_tables(c, prec)["coef"]
    return x, q, o, rphi, rg, far, grids["b"], coef, eps


def _round(a, prec):
    return np.asarray(a, dtype=np.float64 if prec == "fp64" else np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["fp32", "fp32_arith", "fp64"])
def test_bounds_accept_the_rounded_oracle(prec):
    x, q, o, rphi, rg, far, b, coef, eps = _system(prec)
    F = direct.forces(q, rg)
    r_phi, r_g = EW.check(f"cpu-accept-{prec}", _round(rphi, prec), _round(F, prec), q, rphi, rg, far, b, x, o,
                          coef, eps, prec)
    assert r_phi < 0.2 and r_g < 0.2


@pytest.mark.parametrize("prec", ["fp32", "fp32_arith", "fp64"])
def test_bounds_reject_one_bad_potential(prec):
    x, q, o, rphi, rg, far, b, coef, eps = _system(prec)
    F = direct.forces(q, rg)
    bad = rphi.copy()
    bad[17] += 1e-4 * np.sqrt(np.mean(far ** 2))   # one particle off by 1e-4 of the RMS far field
    with pytest.raises(AssertionError, match="phi err/tol"):
        EW.check("cpu-reject-phi", bad, F, q, rphi, rg, far, b, x, o, coef, eps, prec)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_bounds_reject_one_bad_force_component(prec):
    x, q, o, rphi, rg, far, b, coef, eps = _system(prec)
    F = direct.forces(q, rg)
    bad = F.copy()
    bad[5, 1] *= 1.0 + 1e-3
    with pytest.raises(AssertionError, match="grad err/tol"):
        EW.check("cpu-reject-force", rphi, bad, q, rphi, rg, far, b, x, o, coef, eps, prec)


def test_local_bound_rejects_a_shifted_support():
    """Interpolation alone (no global part): one particle interpolated one grid point off."""
    prec = "fp32"
    x, q, o, rphi, rg, far, b, coef, eps = _system(prec)
    phi, g = fast.interpolate(b, np.mod(x, o.L), o)
    xs = x.copy()
    xs[3, 0] += o.h
    phis, gs = fast.interpolate(b, np.mod(xs, o.L), o)
    bad_phi, bad_g = phi.copy(), g.copy()
    bad_phi[3], bad_g[3] = phis[3], gs[3]
    EW.check("cpu-local-accept", _round(phi, prec), _round(g, prec), q, phi, g, phi, b, x, o, coef, eps, prec,
             vec_is_force=False, global_part=False)
    with pytest.raises(AssertionError):
        EW.check("cpu-local-reject", bad_phi, bad_g, q, phi, g, phi, b, x, o, coef, eps, prec,
                 vec_is_force=False, global_part=False)


def test_window_bounds_are_the_fit_tolerance():
    """delta measured on the library's polynomials stays within the fit tolerance (plus the
    sampling margin), and the derivative bound D1 is of the size of the window's slope."""
    x, q, o, rphi, rg, far, b, coef, eps = _system("fp32")
    delta, ddelta, D1, D2 = EW.window_bounds(coef, o)
    assert delta <= 1.25 * EW.fit_tol(eps, "fp32") * 1.01 + 1e-15
    assert 0.1 < D1 < 2.0 and D2 > 0


def test_binding_rejects_wrong_sizes():
    """The binding checks every array's shape against n (or the number of systems) before any
    pointer reaches the library: a short output would be written out of bounds by the kernels."""
    torch = pytest.importorskip("torch")
    pw._expect_shapes(pos=(torch.zeros(4, 3), (4, 3)), q=(torch.zeros(4), (4,)), phi=(None, (4,)))
    for kw in (dict(q=(torch.zeros(3), (4,))), dict(phi=(torch.zeros(5), (4,))),
               dict(force=(torch.zeros(4, 2), (4, 3))), dict(force=(torch.zeros(12), (4, 3))),
               dict(energy=(torch.zeros(2), (1,))), dict(pos=(torch.zeros(4, 3, 1), (4, 3)))):
        with pytest.raises(ValueError, match="must have shape"):
            pw._expect_shapes(**kw)
    # a plan object without a device handle: the shape checks come first, so the wrong sizes
    # are refused even without a GPU
    plan = object.__new__(pw.Plan)
    plan.n_max, plan.dtype, plan._h = 8, torch.float32, None
    pos, q = torch.zeros(4, 3), torch.zeros(4)
    for kw in (dict(phi=torch.zeros(3)), dict(force=torch.zeros(4, 2)), dict(energy=torch.zeros(2))):
        with pytest.raises(ValueError, match="must have shape"):
            plan.compute(pos, q, **kw)
    with pytest.raises(ValueError, match="must have shape"):
        plan.compute(pos, torch.zeros(3))
    with pytest.raises(ValueError, match="must have shape"):
        plan.local(pos, q, phi=torch.zeros(5))
    batch = object.__new__(pw.BatchPlan)
    batch.n_total, batch.nsys, batch.dtype, batch._h = 4, 2, torch.float32, None
    with pytest.raises(ValueError, match="must have shape"):
        batch.compute(pos, q, energy=torch.zeros(1))
    with pytest.raises(ValueError, match="must have shape"):
        batch.compute(pos[:3], q[:3])


def test_chunked_oracle_equals_the_oracle():
    """The worker-process form of Alg. 2 used for n = 1e6 reproduces oracle/fast.py to rounding."""
    import oracle_pool
    x, q, L = W.paper_default(3000, seed=43)
    o = oparams.choose(1e-6, L, m=24)
    p1, g1, gr1 = fast.fast_longrange(x, q, o, return_grids=True)
    p2, g2, gr2 = oracle_pool.fast_longrange(x, q, o, return_grids=True)
    assert np.max(np.abs(p1 - p2)) <= 1e-12 * np.max(np.abs(p1))
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g1))
    # b itself carries the rounding of a's summation order amplified by s_k ~ 1/phihat^2 near
    # the band edge (phihat ~ eps_w ~ 1e-7 there); interpolation multiplies it by phihat again
    assert np.max(np.abs(gr1["b"] - gr2["b"])) <= 1e-9 * np.max(np.abs(gr1["b"]))
    S1 = EW.support_abs_sum(gr1["b"], np.mod(x, o.L), o)
    S2 = oracle_pool.support_abs_sum(gr1["b"], np.mod(x, o.L), o)
    assert np.max(np.abs(S1 - S2)) <= 1e-12 * np.max(S1)
