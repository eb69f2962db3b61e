"""Pins of the oracle's direct Ewald sums (oracle/direct.py)."""
import math

import numpy as np
import pytest

import workloads as W
from conftest import read_table
from oracle import direct
from oracle.pswf import PSWF, split_function


def test_madelung_nacl():
    """Rock-salt cell: phi_i = -q_i M / r0 with the textbook Madelung constant, E = -4 M / r0."""
    M = float(read_table("madelung_nacl.txt")[0][0])
    for a in [1.0, 2.5]:
        x, q, L = W.nacl_cell(a)
        phi, g = direct.total_potential(x, q, L)
        np.testing.assert_allclose(phi, -q * M / (a / 2), rtol=1e-11, atol=0)
        assert abs(direct.energy(q, phi) - (-4.0 * M / (a / 2))) < 1e-10 * 4 * M
        np.testing.assert_allclose(g, 0.0, atol=1e-10)  # every ion is a centre of symmetry


def test_gaussian_ewald_agrees_with_pswf_split():
    """The classical Gaussian split (Example 1) and the PSWF split give the same total potential
    and field (the total does not depend on the split, eq. potential2)."""
    x, q, L = W.paper_default(40, seed=7, L=1.3)
    pg, gg = direct.gauss_ewald(x, q, L)
    pp, gp = direct.total_potential(x, q, L)
    np.testing.assert_allclose(pp, pg, rtol=0, atol=1e-11 * np.max(np.abs(pg)))
    np.testing.assert_allclose(gp, gg, rtol=0, atol=1e-10 * np.max(np.abs(gg)))


def test_split_independence_and_routes():
    """phi_total is the same for different PSWF splits; routes R1 and R2 agree for the
    long-range part of a working split."""
    x, q, L = W.paper_default(60, seed=11)
    t1, g1 = direct.total_potential(x, q, L, rc_o=0.45, cs_o=36.0)
    t2, g2 = direct.total_potential(x, q, L, rc_o=0.3, cs_o=30.0)
    np.testing.assert_allclose(t1, t2, rtol=0, atol=1e-11 * np.max(np.abs(t1)))
    np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-9 * np.max(np.abs(g1)))
    rc, cs = 0.12, 12.0
    r2, _ = direct.longrange_r2(x, q, L, rc, cs, grad=False)
    r2b, _ = direct.longrange_r2(x, q, L, rc, cs, grad=False, rc_o=0.3, cs_o=30.0)
    rms = np.sqrt(np.mean(r2 ** 2))
    assert np.sqrt(np.mean((r2 - r2b) ** 2)) < 1e-12 * rms
    # R1 truncates the Fourier sum at K = 4 K_max; the neglected tail of Mhat decays like
    # |k|^-3 (Lemma 4), so its RMS is a small multiple of the split error e^{-c_s} ~ 6e-6.
    r1, _ = direct.longrange_r1(x, q, L, rc, cs, K=int(4 * cs / (2 * math.pi * rc)), grad=False)
    assert np.sqrt(np.mean((r1 - r2) ** 2)) < 3e-6 * rms


def test_translation_invariance_and_newton():
    """Translating every charge leaves phi unchanged; the exact forces sum to zero."""
    x, q, L = W.paper_default(50, seed=3)
    p0, g0 = direct.total_potential(x, q, L)
    p1, _ = direct.total_potential(np.mod(x + np.array([0.31, -0.77, 0.123]), L), q, L)
    np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-11 * np.max(np.abs(p0)))
    F = direct.forces(q, g0)
    assert np.max(np.abs(F.sum(axis=0))) < 1e-10 * np.max(np.abs(F))


def test_energy_is_quadratic_in_q():
    """E(q) = 1/2 q^T A q, so a central difference in q_i equals phi_i exactly (up to rounding)."""
    x, q, L = W.paper_default(30, seed=5)
    rc, cs = 0.2, 10.0
    K = 12

    def E(qq):
        ph, _ = direct.longrange_r1(x, qq, L, rc, cs, K=K, grad=False)
        return direct.energy(qq, ph)

    ph, _ = direct.longrange_r1(x, q, L, rc, cs, K=K, grad=False)
    for i in [0, 7, 29]:
        d = np.zeros_like(q)
        d[i] = 1e-3
        fd = (E(q + d) - E(q - d)) / 2e-3
        assert abs(fd - ph[i]) < 1e-9 * np.max(np.abs(ph))


def test_scaling_law():
    """Sec. 6.1: phi(x) = phi*(x/L)/L for the same relative split r_c/L."""
    x, q, _ = W.paper_default(30, seed=9)
    p1, g1 = direct.total_potential(x, q, 1.0)
    L = 3.7
    pL, gL = direct.total_potential(x * L, q, L)
    np.testing.assert_allclose(pL, p1 / L, rtol=0, atol=1e-12 * np.max(np.abs(p1)))
    np.testing.assert_allclose(gL, g1 / L ** 2, rtol=0, atol=1e-11 * np.max(np.abs(g1)))


def test_self_term_is_limit_of_mollified_kernel():
    """phi_self = -lim_{r->0} M(r) rho with M = Phi_{r_c}(r)/r (eq. M): compare with M at small r."""
    rc, cs = 0.2, 14.0
    p = PSWF(cs)
    r = 1e-7 * rc
    M0 = float(split_function(r, rc, p)) / r
    assert abs(direct.self_term(np.array([1.0]), rc, cs)[0] + M0) < 1e-6 * M0
    assert abs(M0 - 2.0 / (rc * p.lambda0)) < 1e-6 * M0


def test_local_part_is_compactly_supported():
    """Moving a far-away charge pair (beyond r_c of every target) does not change phi_local."""
    x, q, L = W.paper_default(40, seed=21)
    rc, cs = 0.1, 12.0
    idx = np.arange(10)
    d = np.linalg.norm(direct._min_image(x[idx][:, None, :] - x[None, :, :], L), axis=2)
    far = np.where(np.all(d[:, 10:] > 3 * rc, axis=0))[0] + 10
    assert far.size > 0
    j = far[0]
    x2 = x.copy()
    x2[j] += 0.3 * rc * np.array([1.0, 0.5, -0.2]) / np.linalg.norm([1.0, 0.5, -0.2])
    a, _ = direct.local_direct(x, q, L, rc, cs, target_idx=idx)
    b, _ = direct.local_direct(x2, q, L, rc, cs, target_idx=idx)
    np.testing.assert_array_equal(a, b)
