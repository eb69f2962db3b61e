"""Per-particle parity bounds for potentials and gradients (test infrastructure).

The GPU results are compared with the float64 oracle of Alg. 2 (oracle/fast.py) particle by
particle, not through a norm. With b the oracle's grid after step 4 and S_i the sum of |b_l|
over the P^3 grid points of particle i's support:

  |phi_i - phi_ref,i|          <= 6 g_phi  rms(phi_far)       + (3 delta + 3 u D1 + 4 u) S_i + u |phi_i|
  |d_d phi_i - d_d phi_ref,i|  <= 6 g_grad rms(|grad phi_far|) + (delta' + 3 delta D1 + 3 u (D1 + D2) + 4 u D1) S_i / h

Local part (step 5, eq. FastEwaldSteps34 and eq. force): every grid value enters phi_i times a
product of three window values of size at most 1, each from a fitted polynomial off by at most
delta (so the product by at most ~3 delta), and times the derivative polynomial (off by at most
delta' in units of the grid offset g) for a gradient component, whose chain factor 1/h_d follows.
D1 and D2 bound |phi_1'| and |phi_1''| in grid units: an offset g rounded to the working
precision (error u) moves a window value by u D1 and a derivative by u D2. The float32 grid and
output are rounded once (u S_i, u |phi_i|). delta and delta' are measured on the polynomials the
library evaluates (pswfe_host_tables) against the oracle's window, on a fine grid of offsets.

Global part (steps 1-4): the grid-stage error (spreading, FFT and scaling rounding, the spread's
window fit) reaches phi as a band-limited field sampled at the particles. Its relative l2 size is
bounded by g_phi (g_grad for the gradient), the constants of the whole-pipeline norm bounds
(float32: 2e-6 + 10 delta for phi, 2e-5 + 100 delta for the gradient; float64: 1e-11 + 10 delta
and 1e-10 + 100 delta). Over n samples the largest value of such a field stays below about
sqrt(2 ln n) (<= 5.3 for n <= 1e6) times its RMS: 6 is allowed. A single particle whose support,
offset or window were wrong would be off by O(|phi_i|) and fail.

The float32 arithmetic path (fp32_arith) also rounds inside the interpolation sums: the local
rounding term grows from 4 u S_i to (4 + P/2 + P^2/16 + 4) u S_i (recursive summation bounds
the error of a sum of k terms by about k u times the sum of their magnitudes); its grid stage
is within the same norm bounds as the float32 path's.

Each check returns the largest err/tol ratio and records it for the session summary.
"""
from __future__ import annotations

import numpy as np

from oracle import fast
from oracle.pswf import PSWF, window_1d, window_1d_deriv

U = {"fp32": 6e-8, "fp32_arith": 6e-8, "fp64": 1.2e-16}
RATIOS: list[tuple[str, float]] = []


def fit_tol(eps, prec):
    return max(0.01 * eps, 1e-15 if prec == "fp64" else 5e-9)


def global_rel(eps, prec):
    """(g_phi, g_grad): relative l2 bounds of the grid-stage error reaching phi and grad phi."""
    d = fit_tol(eps, prec)
    if prec != "fp64":
        return 2e-6 + 10 * d, 2e-5 + 100 * d
    return 1e-11 + 10 * d, 1e-10 + 100 * d


def window_bounds(coef, o):
    """(delta, delta', D1, D2) for the library's window polynomials `coef` (P, deg + 1) against
    the oracle's phi_1: the largest value and derivative fit errors in grid units, and bounds
    on |phi_1'| and |phi_1''| in grid units."""
    P = o.P
    pw_ = PSWF(o.cw)
    g = np.linspace(-0.5, 0.5, 1601)
    dv_max = ddv_max = d1 = d2 = 0.0
    for j in range(P):
        s = 2 * (g + (P - 1) / 2 - j) / P
        c = coef[j][::-1]
        v = np.polyval(c, g)
        dv = np.polyval(np.polyder(c), g)
        ddv = np.polyval(np.polyder(c, 2), g)
        ref = window_1d(s, pw_)
        dref = window_1d_deriv(np.clip(s, -1, 1), pw_) * 2 / P
        dv_max = max(dv_max, float(np.max(np.abs(v - ref))))
        ddv_max = max(ddv_max, float(np.max(np.abs(dv - dref))))
        d1 = max(d1, float(np.max(np.abs(dv))))
        d2 = max(d2, float(np.max(np.abs(ddv))))
    # the sampled maxima of the errors, with a margin for the points between samples
    return 1.25 * dv_max + 1e-16, 1.25 * ddv_max + 1e-15, d1, d2


def support_abs_sum(b_xyz, x, o, chunk=200_000):
    """S_i = sum over the P^3 support points of particle i of |b_l| (b in oracle order [x, y, z])."""
    m, P = o.m, o.P
    bf = np.abs(np.asarray(b_xyz, dtype=np.float64)).reshape(-1)
    out = np.zeros(len(x))
    for s in range(0, len(x), chunk):
        idx, _, _ = fast.support(np.mod(x[s:s + chunk], o.L), o)
        acc = np.zeros(idx.shape[0])
        for jx in range(P):
            for jy in range(P):
                base = (idx[:, 0, jx] * m + idx[:, 1, jy]) * m
                acc += bf[base[:, None] + idx[:, 2, :]].sum(axis=1)
        out[s:s + chunk] = acc
    return out


def check(name, phi, vec, q, ref_phi, ref_grad, far, b_xyz, x, o, coef, eps, prec, *, vec_is_force=True,
          global_part=True, idx=None):
    """Asserts the per-particle bounds above for phi (n) and vec (n, 3) against the oracle's
    phi (far field plus self term) and grad phi; vec is the force -q grad phi (or grad phi with
    vec_is_force=False). far: the oracle's far field on the same particles (its RMS scales the
    global part). idx: the particles compared, when only a sample is (x and q are then the full
    system's, phi, vec, ref_*, far those of the sample). Returns (max ratio phi, max ratio grad)."""
    u = U[prec]
    # rounding of the interpolation sums, in units of u times S_i: a float64 sum rounded once to
    # float32 (4); with float32 arithmetic the recursive sums themselves (an x-line of P terms in two
    # accumulators, about P^2 / 16 lines per lane, 4 levels of the 16-lane reduction) add
    # P / 2 + P^2 / 16 + 4 more
    r_sum = 4 + ((o.P / 2 + o.P ** 2 / 16 + 4) if prec == "fp32_arith" else 0)
    delta, ddelta, D1, D2 = window_bounds(coef, o)
    xs = x if idx is None else x[idx]
    qs = q if idx is None else q[idx]
    if len(xs) > 100_000:   # large systems: the same sums over particle chunks in worker processes
        import oracle_pool
        S = oracle_pool.support_abs_sum(b_xyz, xs, o)
    else:
        S = support_abs_sum(b_xyz, xs, o)
    g_phi, g_grad = global_rel(eps, prec) if global_part else (0.0, 0.0)
    ref_phi = np.asarray(ref_phi, dtype=np.float64)
    rms_phi = float(np.sqrt(np.mean(np.asarray(far, dtype=np.float64) ** 2))) if len(far) else 0.0
    tol_phi = 6 * g_phi * rms_phi + (3 * delta + 3 * u * D1 + r_sum * u) * S + u * np.abs(ref_phi) + 1e-300
    err_phi = np.abs(np.asarray(phi, dtype=np.float64) - ref_phi)
    r_phi = float(np.max(err_phi / tol_phi)) if len(err_phi) else 0.0
    r_g = 0.0
    if vec is not None:
        ref_g = np.asarray(ref_grad, dtype=np.float64)
        rms_g = float(np.sqrt(np.mean(np.sum(ref_g ** 2, axis=1)))) if len(ref_g) else 0.0
        tol_g = (6 * g_grad * rms_g + (ddelta + 3 * delta * D1 + 3 * u * (D1 + D2) + r_sum * u * D1) * S / o.h
                 + u * np.max(np.abs(ref_g), axis=1) + 1e-300)
        v = np.asarray(vec, dtype=np.float64)
        if vec_is_force:   # F = -q grad phi: the bound scales with |q_i|
            err_g = np.abs(v + qs[:, None] * ref_g)
            tol_g = np.abs(qs) * tol_g + 1e-300
        else:
            err_g = np.abs(v - ref_g)
        r_g = float(np.max(err_g / tol_g[:, None])) if len(err_g) else 0.0
    RATIOS.append((name, max(r_phi, r_g)))
    assert r_phi <= 1.0, f"{name}: phi err/tol {r_phi:.3g}"
    assert r_g <= 1.0, f"{name}: grad err/tol {r_g:.3g}"
    return r_phi, r_g
