"""Pins of the cuboid-box oracle (oracle/variants.py with per-axis sides and grid sizes; Sec. 6.1,
remark on cuboid domains):

* a box doubled along one axis, holding the system twice (x and x + L e_a), is the same periodic
  system: its potentials equal the cube's, both for the direct Fourier sum and for Alg. 2 on the
  doubled grid (same spacing);
* on a genuine cuboid (unequal sides, unequal spacings) Alg. 2 meets eps against the direct sum;
* the library's box parameter rule agrees with the oracle's.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import params as oparams
from oracle import variants as V


def _cube(eps=1e-8, n=120, seed=5, rc=0.2):
    x, q, L = W.paper_default(n, seed=seed)
    p = oparams.choose(eps, L, rc=rc)
    return x, q, L, V.VariantParams(L, p.rc, p.cs, p.m, p.P)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_doubled_box_is_the_cube(axis):
    x, q, L, vp = _cube()
    shift = np.zeros(3)
    shift[axis] = L
    x2, q2 = np.concatenate([x, x + shift]), np.concatenate([q, q])
    sides = [L, L, L]
    grids = [vp.m, vp.m, vp.m]
    sides[axis] *= 2
    grids[axis] *= 2
    vp2 = V.VariantParams(sides[0], vp.rc, vp.cs, grids[0], vp.P, Ly=sides[1], Lz=sides[2], my=grids[1],
                          mz=grids[2])
    a, ga = V.fast_variant(x, q, vp)
    b, gb = V.fast_variant(x2, q2, vp2)
    n = len(q)
    assert np.max(np.abs(b[:n] - a)) < 1e-11 * np.max(np.abs(a))
    assert np.max(np.abs(b[n:] - a)) < 1e-11 * np.max(np.abs(a))
    assert np.max(np.abs(gb[:n] - ga)) < 1e-10 * np.max(np.abs(ga))
    K = V.reference_modes(vp) // 3
    da, _ = V.far_direct_variant(x, q, vp, K)
    db, _ = V.far_direct_variant(x2, q2, vp2, K)
    assert np.max(np.abs(db[:n] - da)) < 1e-11 * np.max(np.abs(da))


@pytest.mark.parametrize("sides,split", [((1.0, 1.3, 0.8), "pswf"), ((0.9, 1.5, 1.2), "pswf"),
                                         ((1.0, 1.3, 0.8), "gauss")])
def test_cuboid_fast_meets_eps(sides, split):
    eps = 1e-6
    rng = np.random.Generator(np.random.PCG64(77))
    n = 200
    x = rng.uniform(0, 1, (n, 3)) * np.asarray(sides)
    q = rng.standard_normal(n)
    q -= q.mean()
    vp = V.box_params(eps, sides, rc=0.12)
    assert vp.grids[0] != vp.grids[1] != vp.grids[2]
    if split == "gauss":   # Gaussian split, same r_c and c_s = log(1/eps), a finer grid and support
        vp = V.VariantParams(vp.L, vp.rc, math.log(1 / eps), 2 * vp.m, vp.P + 4, split="gauss", Ly=vp.Ly,
                             Lz=vp.Lz, my=2 * vp.my, mz=2 * vp.mz)
    ref, gref = V.far_direct_variant(x, q, vp, V.reference_modes(vp), grad=True)
    phi, g = V.fast_variant(x, q, vp)
    far = ref + V.self_coefficient(vp) * q
    assert np.linalg.norm(phi - ref) / np.linalg.norm(far) < eps
    assert np.linalg.norm(g - gref) / np.linalg.norm(gref) < 30 * eps


def test_box_params_match_library():
    pw = pytest.importorskip("paper_2602_16591_amd")
    for sides, eps, rc in [((1.0, 1.3, 0.8), 1e-6, 0.12), ((2.0, 1.0, 1.0), 1e-10, 0.2), ((1.0, 1.0, 1.0), 1e-6, 0.1)]:
        o = V.box_params(eps, sides, rc=rc)
        c = pw.choose_params_box(eps, sides, rc=rc)
        assert (c.m, c.my, c.mz, c.P) == tuple(o.grids) + (o.P,)
        assert abs(c.cs - o.cs) < 1e-12 * o.cs and abs(c.rc - o.rc) < 1e-14
        assert (c.L, c.Ly, c.Lz) == sides
    cube = pw.choose_params(1e-6, 1.0, rc=0.1)
    box = pw.choose_params_box(1e-6, (1.0, 1.0, 1.0), rc=0.1)
    assert (cube.m, cube.P, cube.cs) == (box.m, box.P, box.cs)
