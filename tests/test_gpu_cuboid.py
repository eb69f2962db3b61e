"""GPU parity on cuboid boxes (Sec. 6.1, remark on cuboid domains): unequal sides and grid
sizes, against the float64 oracle's Alg. 2 on the same box (oracle/variants.py), the identity of a
box doubled along one axis with the cube (far field and the full Ewald sum), and batches that mix
cubes and cuboids."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct
from oracle import params as oparams
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


def box_system(sides, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0, 1, (n, 3)) * np.asarray(sides)
    q = rng.standard_normal(n)
    return x, q - q.mean()


def with_split(c, split, window, cs, m_factor=1, P_add=0):
    """A copy of cuboid parameters with another split/window (the cuboid form of a comparison
    configuration)."""
    c2 = type(c).from_buffer_copy(c)
    c2.split, c2.window, c2.cs = pw.SPLITS[split], pw.WINDOWS[window], cs
    c2.m, c2.my, c2.mz, c2.P = c.m * m_factor, c.my * m_factor, c.mz * m_factor, c.P + P_add
    c2.h = c2.L / c2.m
    c2.alpha = 0.5 * c2.P * c2.h
    c2.cw = 0.5 * math.pi * c2.P
    if window == "gauss":
        c2.cg = V.gauss_window_shape(c2.P)
    return c2


CASES = [
    # (name, sides, eps, rc, precisions, split/window change)
    ("box_1_1.3_0.8", (1.0, 1.3, 0.8), 1e-6, 0.12, ("fp64", "fp32"), None),
    ("box_0.9_1.5_1.2", (0.9, 1.5, 1.2), 1e-6, 0.15, ("fp64", "fp32"), None),
    ("box_tight_fp64", (1.0, 0.7, 1.6), 1e-10, 0.14, ("fp64",), None),
    ("box_gauss_split", (1.0, 1.3, 0.8), 1e-6, 0.12, ("fp64", "fp32"), ("gauss", "gauss")),
    ("box_bspline", (1.0, 1.3, 0.8), 1e-5, 0.12, ("fp64",), ("pswf", "bspline")),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_cuboid_matches_oracle(case, prec):
    _, sides, eps, rc, precs, change = case
    if prec not in precs:
        pytest.skip("precision not used for this case")
    x, q = box_system(sides, 3000, seed=81)
    if prec == "fp32":
        x, q = x.astype(np.float32).astype(np.float64), q.astype(np.float32).astype(np.float64)
    c = pw.choose_params_box(eps, sides, rc=rc)
    vp = V.box_params(eps, sides, rc=rc)
    assert (c.m, c.my, c.mz, c.P) == tuple(vp.grids) + (vp.P,)
    if change is not None:
        split, window = change
        cs = math.log(1.0 / eps)
        c = with_split(c, split, window, cs, m_factor=2 if split == "gauss" else 1, P_add=4 if split == "gauss" else 0)
        vp = V.VariantParams(vp.L, vp.rc, cs, c.m, c.P, split=split, window=window, cg=c.cg, Ly=vp.Ly, Lz=vp.Lz,
                             my=c.my, mz=c.mz)
    plan = pw.Plan(c, prec, n_max=len(q))
    phi, F, E = plan.compute(tdev(x, prec), tdev(q, prec))
    rphi, rg = V.fast_variant(x, q, vp)
    far = rphi + V.self_coefficient(vp) * q
    tol_phi = (1e-11 if prec == "fp64" else 2e-6) + 10 * fit_tol(eps, prec)
    tol_F = (1e-10 if prec == "fp64" else 2e-5) + 100 * fit_tol(eps, prec)
    assert np.linalg.norm(phi.double().cpu().numpy() - rphi) / np.linalg.norm(far) < tol_phi
    rF = direct.forces(q, rg)
    assert np.linalg.norm(F.double().cpu().numpy() - rF) / np.linalg.norm(rF) < tol_F
    Eref = 0.5 * float(q @ rphi)
    assert abs(float(E.cpu()[0]) - Eref) <= tol_phi * 0.5 * float(np.abs(q) @ np.abs(far)) + 1e-12 * abs(Eref)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_doubled_box_equals_cube(axis):
    """The cube's system placed twice in a box doubled along one axis (grid doubled too): far
    field, forces and the full Ewald sum (with the real-space residual on per-axis cells) equal the
    cube's at every copy."""
    x, q, L = W.paper_default(700, seed=82)
    c = pw.choose_params(1e-10, L, rc=0.2)
    shift = np.zeros(3)
    shift[axis] = L
    x2, q2 = np.concatenate([x, x + shift]), np.concatenate([q, q])
    c2 = type(c).from_buffer_copy(c)
    sides, grids = [L, L, L], [c.m, c.m, c.m]
    sides[axis] *= 2
    grids[axis] *= 2
    c2.L, c2.Ly, c2.Lz = sides
    c2.m, c2.my, c2.mz = grids
    c2.h = c2.L / c2.m
    c2.alpha = 0.5 * c2.P * c2.h
    n = len(q)
    for total in (False, True):
        p1 = pw.Plan(c, "fp64", n_max=n)
        p2 = pw.Plan(c2, "fp64", n_max=2 * n)
        a, Fa, Ea = p1.compute(tdev(x, "fp64"), tdev(q, "fp64"), total=total)
        b, Fb, Eb = p2.compute(tdev(x2, "fp64"), tdev(q2, "fp64"), total=total)
        a, b, Fa, Fb = a.cpu().numpy(), b.cpu().numpy(), Fa.cpu().numpy(), Fb.cpu().numpy()
        sc = np.max(np.abs(a))
        assert np.max(np.abs(b[:n] - a)) < 1e-11 * sc and np.max(np.abs(b[n:] - a)) < 1e-11 * sc
        assert np.max(np.abs(Fb[:n] - Fa)) < 1e-10 * np.max(np.abs(Fa))
        assert abs(float(Eb.cpu()[0]) - 2 * float(Ea.cpu()[0])) < 1e-10 * abs(float(Ea.cpu()[0]))


@pytest.mark.parametrize("yz", ["1", "0"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_mixes_cubes_and_cuboids(prec, yz, monkeypatch):
    """A batch of cubes and cuboids against one plan per system; yz=1 runs the batch's y and z
    FFT passes and the scaling fused per spectrum column (on cuboid planes), against the
    separate passes of the single-system plans."""
    systems = [((1.0, 1.3, 0.8), 1500, 83), ((1.0, 1.0, 1.0), 900, 84), ((0.9, 1.5, 1.2), 2000, 85)]
    params, xs, qs = [], [], []
    for sides, n, seed in systems:
        x, q = box_system(sides, n, seed)
        if prec == "fp32":
            x, q = x.astype(np.float32).astype(np.float64), q.astype(np.float32).astype(np.float64)
        params.append(pw.choose_params_box(1e-6, sides, rc=0.15))
        xs.append(x)
        qs.append(q)
    counts = [len(q) for q in qs]
    monkeypatch.setenv("PSWFE_YZ_FFT", yz)
    plan = pw.BatchPlan(params, counts, prec)
    monkeypatch.setenv("PSWFE_YZ_FFT", "0")
    phi, F, E = plan.compute(tdev(np.concatenate(xs), prec), tdev(np.concatenate(qs), prec), total=True)
    lphi, lF, lE = plan.split(phi.cpu().numpy()), plan.split(F.cpu().numpy()), E.cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-6
    for k in range(3):
        single = pw.Plan(params[k], prec, n_max=counts[k])
        sp, sF, sE = single.compute(tdev(xs[k], prec), tdev(qs[k], prec), total=True)
        assert np.linalg.norm(lphi[k] - sp.cpu().numpy()) <= tol * np.linalg.norm(sp.cpu().numpy())
        assert np.linalg.norm(lF[k] - sF.cpu().numpy()) <= tol * np.linalg.norm(sF.cpu().numpy())
        assert abs(lE[k] - float(sE.cpu()[0])) <= tol * abs(lE[k])
