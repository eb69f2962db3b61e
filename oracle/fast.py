"""Oracle: fast Fourier-space summation (Alg. 2) in float64, step by step.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Steps in the paper's order (Alg. 2, eqs. spread_def, diag_scale, FastEwaldSteps34, force):
  1. spread   a_l = sum_j rho_j phitilde(x_j - h l), over the P^3 grid points of the support
  2. FFT      ahat_k = sum_l a_l e^{+2 pi i k.l/m}
  3. scale    bhat_k = s_k ahat_k,  bhat_0 = 0
  4. IFFT     b_l = sum_k bhat_k e^{-2 pi i k.l/m}
  5. interpolate  phi_i = sum_l b_l phitilde(x_i - h l),  grad phi_i = sum_l b_l grad phitilde
then the self term (Sec. 3.1) is added: the result is phi_far + phi_self.

The window is phi(x) = prod_d phi_1(x_d/alpha) with phi_1 = psi_0^{c_w}/psi_0^{c_w}(0) on [-1, 1]
(Sec. 4.3), evaluated here from the Legendre series (no polynomial approximation).

Readings taken where the paper is silent (listed in the design notes):
  * DFT normalisation: with the unnormalised transform pair of steps 2 and 4,
        s_k = h^6 Mhat(k) / (V phihat(k)^2),
    where phihat is the continuous transform of Table 2; the paper's eq. diag_scale omits
    the h^6 that the Riemann sums of steps 1-2 and 4-5 introduce.
  * Ball truncation (``ball=True``): modes with |k| > m/2 (the corners of the cube I_m) are
    set to zero. Their true contribution is bounded by the split-error tail of Prop. 1, but
    s_k there is ~1e10-1e13 times its in-ball size and amplifies rounding errors.
  * Support points: the P points l = floor(x/h - P/2) + 1 + j, j = 0..P-1, per dimension
    (the window is evaluated on [-1, 1); its value psi_0(1)/psi_0(0) at +-1 is ~eps_w).
"""
from __future__ import annotations

import math

import numpy as np

from .params import Params
from .pswf import PSWF, gammahat, window_1d, window_1d_deriv, window_hat_1d
from .direct import self_term


def support(x: np.ndarray, p: Params):
    """Grid indices (mod m) and window values/derivatives for each particle and dimension.

    Returns idx (n, 3, P) int, w (n, 3, P), dw (n, 3, P) with dw = d/dx_d of phi_1((x_d - h l)/alpha).
    """
    pw = PSWF(p.cw)
    h = p.h
    t = x / h                                              # (n, 3) grid units
    start = np.floor(t - p.P / 2.0).astype(np.int64) + 1
    l = start[:, :, None] + np.arange(p.P)[None, None, :]  # (n, 3, P)
    s = (x[:, :, None] - h * l) / p.alpha                  # window argument (x - h l)/alpha
    w = window_1d(s, pw)
    dw = window_1d_deriv(s, pw) / p.alpha
    return np.mod(l, p.m), w, dw


def spread(x: np.ndarray, q: np.ndarray, p: Params) -> np.ndarray:
    """Step 1: a[lx, ly, lz] = sum_j q_j phi_1(.)phi_1(.)phi_1(.) (eq. spread_def)."""
    m, P = p.m, p.P
    idx, w, _ = support(x, p)
    a = np.zeros(m ** 3)
    for jx in range(P):
        for jy in range(P):
            wxy = q * w[:, 0, jx] * w[:, 1, jy]
            base = (idx[:, 0, jx] * m + idx[:, 1, jy]) * m
            flat = (base[:, None] + idx[:, 2, :]).ravel()
            a += np.bincount(flat, weights=(wxy[:, None] * w[:, 2, :]).ravel(), minlength=m ** 3)
    return a.reshape(m, m, m)


def kvec(m: int) -> np.ndarray:
    """Integer wave numbers of FFT bins 0..m-1 in I_m (Sec. 2.1): {-m/2, ..., m/2-1} for even m,
    {-(m-1)/2, ..., (m-1)/2} for odd m."""
    i = np.arange(m)
    return np.where(i <= (m - 1) // 2, i, i - m)


def scaling(p: Params, ball: bool = True) -> np.ndarray:
    """s_k = h^6 Mhat(k) / (V phihat(k)^2) on the m^3 FFT bins; s_0 = 0 (Alg. 2 step 3).

    With ``ball`` the modes outside the mollifier's band, 2 pi |k| / L > c_s / r_c, are set to
    zero; with the grid tied to the band (eq. csrc) this is the ball |k| <= m/2."""
    m, L = p.m, p.L
    V = L ** 3
    h = p.h
    ps, pw = PSWF(p.cs), PSWF(p.cw)
    k = kvec(m)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    # Mhat(k) = L^2 gammahat(2 pi |k| / L) / (pi |k|^2)  (eq. Fsum, eq. MhatPSWF)
    k2max = int(k2.max())
    kn = np.sqrt(np.arange(k2max + 1, dtype=np.float64))
    Mtab = np.zeros(k2max + 1)
    Mtab[1:] = L * L / (math.pi * kn[1:] ** 2) * gammahat(2.0 * math.pi * kn[1:] / L, p.rc, ps)
    Mhat = Mtab[k2]
    ph1 = window_hat_1d(2.0 * math.pi * k / L, p.alpha, pw)            # (m,)
    phihat = ph1[:, None, None] * ph1[None, :, None] * ph1[None, None, :]
    s = h ** 6 * Mhat / (V * phihat ** 2)
    s[0, 0, 0] = 0.0
    if ball:
        kband = p.cs * L / (2.0 * math.pi * p.rc)           # omega = c_s / r_c  (eq. csrc)
        s[k2 > kband * kband * (1.0 + 1e-12)] = 0.0
    return s


def interpolate(b: np.ndarray, x: np.ndarray, p: Params, grad: bool = True):
    """Step 5 (eq. FastEwaldSteps34) and its gradient (eq. force)."""
    m, P = p.m, p.P
    idx, w, dw = support(x, p)
    n = x.shape[0]
    phi = np.zeros(n)
    g = np.zeros((n, 3)) if grad else None
    bf = b.reshape(-1)
    for jx in range(P):
        for jy in range(P):
            base = (idx[:, 0, jx] * m + idx[:, 1, jy]) * m
            vals = bf[base[:, None] + idx[:, 2, :]]                 # (n, P) over z
            sz = np.einsum("np,np->n", vals, w[:, 2, :])
            phi += w[:, 0, jx] * w[:, 1, jy] * sz
            if grad:
                dz = np.einsum("np,np->n", vals, dw[:, 2, :])
                g[:, 0] += dw[:, 0, jx] * w[:, 1, jy] * sz
                g[:, 1] += w[:, 0, jx] * dw[:, 1, jy] * sz
                g[:, 2] += w[:, 0, jx] * w[:, 1, jy] * dz
    return phi, g


def fast_longrange(x, q, p: Params, ball: bool = True, grad: bool = True, return_grids: bool = False):
    """phi_far + phi_self (and grad phi_far) by Alg. 2 in float64."""
    x = np.mod(np.asarray(x, dtype=np.float64), p.L)
    q = np.asarray(q, dtype=np.float64)
    a = spread(x, q, p)                                  # step 1
    m3 = p.m ** 3
    ahat = np.fft.ifftn(a) * m3                          # step 2: e^{+2 pi i k.l/m}, unnormalised
    s = scaling(p, ball=ball)
    bhat = s * ahat                                      # step 3
    b = np.fft.fftn(bhat).real                           # step 4: e^{-2 pi i k.l/m}, unnormalised
    phi, g = interpolate(b, x, p, grad=grad)             # step 5
    phi = phi + self_term(q, p.rc, p.cs)
    if return_grids:
        return phi, g, dict(a=a, ahat=ahat, s=s, b=b)
    return phi, g
