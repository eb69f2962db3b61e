"""Oracle: the comparison splits and windows of Sec. 4.3.1 and Sec. 7.3.1-7.4, run through Alg. 2.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper compares its PSWF split and PSWF window with the classical alternatives:

* Splits (Sec. 3.1, Example 1). Both give Mhat(w) = 4 pi gammahat(w) / w^2:
    - PSWF: gammahat from eq. PSWF_mollifier_ft (``pswf.gammahat``), band limited to
      |w| <= c_s / r_c; self term -2 rho / (r_c lambda_0(c_s)).
    - Gaussian: gammahat(w) = exp(-sigma^2 w^2 / 4), no band limit; self term
      -2 rho / (sqrt(pi) sigma). The comparisons match the truncation levels by
      c_s = (r_c / sigma)^2 (eq. directsumexample), so sigma = r_c / sqrt(c_s).
* Windows (Table 2), per dimension, with alpha = P h / 2:
    - PSWF: psi_0^{c_w}(x/alpha) / psi_0^{c_w}(0), c_w = pi P / 2 (eq. cwP);
    - Gaussian: exp(-c_g (x/alpha)^2) truncated to |x| <= alpha, deconvolved with its
      free-space transform alpha sqrt(pi/c_g) exp(-w^2 alpha^2 / (4 c_g)) (the common practice
      the paper describes);
    - cardinal B-spline of order P: B_P(x/h), the (P-1)-fold convolution of the unit box
      B_1 = 1 on [-1/2, 1/2), support P points; deconvolved with the SPME scaling (Sec. 7.1):
      the transform h B_P^(h w) is replaced by its periodisation over the grid's aliases,
      h sum_p B_P^(h w + 2 pi p), which by Poisson summation is the discrete transform of the
      spline's integer samples, h sum_j B_P(j) e^{-i h w j}.

Alg. 2 is then the same five steps as ``fast.fast_longrange``:
    s_k = h^6 Mhat(k) / (V prod_d phihat_d(k_d)^2),
with the modes outside a ball set to zero: the PSWF split's band |k| <= c_s L / (2 pi r_c), as
in ``fast.scaling``; for the Gaussian split, which has no band, |k| <= m/2 (beyond it the
corners of the grid's cube of modes multiply rounding errors by up to 1/phihat^2 in all three
dimensions at once).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .pswf import PSWF, gammahat, window_1d, window_1d_deriv, window_hat_1d
from .direct import structure_factor, _exp_tables

SPLITS = ("pswf", "gauss")
WINDOWS = ("pswf", "gauss", "bspline")


@dataclass
class VariantParams:
    L: float
    rc: float
    cs: float          # PSWF bandlimit, or (r_c / sigma)^2 for the Gaussian split
    m: int
    P: int
    split: str = "pswf"
    window: str = "pswf"
    cg: float = 0.0    # Gaussian window shape (window == "gauss")

    @property
    def h(self) -> float:
        return self.L / self.m

    @property
    def alpha(self) -> float:
        return self.P * self.h / 2.0

    @property
    def cw(self) -> float:
        return math.pi * self.P / 2.0

    @property
    def sigma(self) -> float:
        return self.rc / math.sqrt(self.cs)


def gauss_window_shape(P: int) -> float:
    """Default Gaussian window shape c_g for support P (a reading; the paper does not state it):
    c_g = 0.8 * pi P / 2, i.e. 0.8 times the PSWF window's bandlimit c_w = pi P / 2. Measured with
    this oracle at the (m, P) of Table 3's Gaussian/Gaussian column (eps = 1e-4, 1e-6, 1e-8),
    the error is smallest for c_g / c_w between 0.7 and 0.9."""
    return 0.8 * math.pi * P / 2.0


# ---------------------------------------------------------------------------------------
# Windows
# ---------------------------------------------------------------------------------------

def bspline(x, P: int):
    """Centred cardinal B-spline B_P(x) (Table 2): B_1 is the unit box on
    [-1/2, 1/2) and B_{P} = B_{P-1} * B_1. Evaluated by the two-term recurrence that the
    convolution gives, B_P(x) = ((P/2 + x) B_{P-1}(x + 1/2) + (P/2 - x) B_{P-1}(x - 1/2)) / (P - 1)."""
    x = np.asarray(x, dtype=np.float64)
    # order k holds B_k(x + c) at the shifts c = -(P - k)/2 + i, i = 0..P-k, the arguments that
    # B_P(x) needs from it
    vals = [np.where((x + c >= -0.5) & (x + c < 0.5), 1.0, 0.0) for c in (-(P - 1) / 2.0 + i for i in range(P))]
    for k in range(2, P + 1):
        nxt = []
        for i in range(P - k + 1):
            y = x + (-(P - k) / 2.0 + i)
            nxt.append(((k / 2.0 + y) * vals[i + 1] + (k / 2.0 - y) * vals[i]) / (k - 1))
        vals = nxt
    return vals[0]


def bspline_deriv(x, P: int):
    """d/dx B_P(x) = B_{P-1}(x + 1/2) - B_{P-1}(x - 1/2) (derivative of the convolution with the box)."""
    x = np.asarray(x, dtype=np.float64)
    return bspline(x + 0.5, P - 1) - bspline(x - 0.5, P - 1)


def bspline_hat(omega, h: float, P: int):
    """Transform of x -> B_P(x/h): h (sin(h w / 2) / (h w / 2))^P (Table 2)."""
    u = 0.5 * h * np.asarray(omega, dtype=np.float64)
    return h * np.sinc(u / math.pi) ** P


def spme_factor(k, m: int, P: int):
    """sum_j B_P(j) e^{-2 pi i k j / m} over the integers j inside the support (real: B_P is even)."""
    k = np.asarray(k, dtype=np.float64)
    j = np.arange(-(P // 2), P // 2 + 1)
    bj = bspline(j.astype(np.float64), P)
    return np.cos(2.0 * math.pi * np.multiply.outer(k, j) / m) @ bj


def gauss_window(s, cg: float):
    """exp(-c_g s^2) on [-1, 1], 0 outside (s = x / alpha)."""
    s = np.asarray(s, dtype=np.float64)
    return np.where(np.abs(s) <= 1.0, np.exp(-cg * s * s), 0.0)


def gauss_window_deriv(s, cg: float):
    s = np.asarray(s, dtype=np.float64)
    return np.where(np.abs(s) <= 1.0, -2.0 * cg * s * np.exp(-cg * s * s), 0.0)


def gauss_window_hat(omega, alpha: float, cg: float):
    """Free-space transform of x -> exp(-c_g (x/alpha)^2): alpha sqrt(pi/c_g) exp(-w^2 alpha^2/(4 c_g))."""
    w = np.asarray(omega, dtype=np.float64)
    return alpha * math.sqrt(math.pi / cg) * np.exp(-w * w * alpha * alpha / (4.0 * cg))


def window_values(d, vp: VariantParams):
    """Window and its x-derivative at offsets d = x - h l (any shape)."""
    if vp.window == "pswf":
        pw = PSWF(vp.cw)
        s = d / vp.alpha
        return window_1d(s, pw), window_1d_deriv(s, pw) / vp.alpha
    if vp.window == "gauss":
        s = d / vp.alpha
        return gauss_window(s, vp.cg), gauss_window_deriv(s, vp.cg) / vp.alpha
    if vp.window == "bspline":
        u = d / vp.h
        return bspline(u, vp.P), bspline_deriv(u, vp.P) / vp.h
    raise ValueError(vp.window)


def window_hat(k, vp: VariantParams):
    """phihat_d at integer wave numbers k (the deconvolution factor of each dimension)."""
    omega = 2.0 * math.pi * np.asarray(k, dtype=np.float64) / vp.L
    if vp.window == "pswf":
        return window_hat_1d(omega, vp.alpha, PSWF(vp.cw))
    if vp.window == "gauss":
        return gauss_window_hat(omega, vp.alpha, vp.cg)
    if vp.window == "bspline":
        return vp.h * spme_factor(k, vp.m, vp.P)
    raise ValueError(vp.window)


# ---------------------------------------------------------------------------------------
# Splits
# ---------------------------------------------------------------------------------------

def mhat(omega, vp: VariantParams):
    """Mhat(w) = 4 pi gammahat(w) / w^2 for w > 0."""
    w = np.asarray(omega, dtype=np.float64)
    if vp.split == "pswf":
        g = gammahat(w, vp.rc, PSWF(vp.cs))
    elif vp.split == "gauss":
        g = np.exp(-vp.sigma ** 2 * w * w / 4.0)
    else:
        raise ValueError(vp.split)
    return 4.0 * math.pi * g / (w * w)


def self_coefficient(vp: VariantParams) -> float:
    """lim_{r->0} M(r): 2 / (r_c lambda_0(c_s)) for the PSWF split, 2 / (sqrt(pi) sigma) for the Gaussian."""
    if vp.split == "pswf":
        return 2.0 / (vp.rc * PSWF(vp.cs).lambda0)
    return 2.0 / (math.sqrt(math.pi) * vp.sigma)


def band_edge(vp: VariantParams) -> float:
    """Largest |k| kept: the PSWF split's band edge c_s L / (2 pi r_c), or m/2 for the Gaussian split."""
    if vp.split == "pswf":
        return vp.cs * vp.L / (2.0 * math.pi * vp.rc)
    return vp.m / 2.0


# ---------------------------------------------------------------------------------------
# Alg. 2 with a chosen split and window
# ---------------------------------------------------------------------------------------

def kvec(m: int) -> np.ndarray:
    i = np.arange(m)
    return np.where(i <= (m - 1) // 2, i, i - m)


def support(x, vp: VariantParams):
    """Per particle and dimension: the P grid indices (mod m) l = floor(x/h - P/2) + 1 + j and the
    window values and derivatives at x - h l."""
    t = x / vp.h
    start = np.floor(t - vp.P / 2.0).astype(np.int64) + 1
    l = start[:, :, None] + np.arange(vp.P)[None, None, :]
    w, dw = window_values(x[:, :, None] - vp.h * l, vp)
    return np.mod(l, vp.m), w, dw


def scaling(vp: VariantParams) -> np.ndarray:
    m, L, h = vp.m, vp.L, vp.h
    k = kvec(m)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    kn = np.sqrt(np.arange(int(k2.max()) + 1, dtype=np.float64))
    mt = np.zeros(kn.size)
    mt[1:] = mhat(2.0 * math.pi * kn[1:] / L, vp)
    ph = window_hat(k, vp)
    phihat = ph[:, None, None] * ph[None, :, None] * ph[None, None, :]
    s = h ** 6 * mt[k2] / (L ** 3 * phihat ** 2)
    s[0, 0, 0] = 0.0
    kb = band_edge(vp)
    s[k2 > kb * kb * (1.0 + 1e-12)] = 0.0
    return s


def fast_variant(x, q, vp: VariantParams, grad: bool = True):
    """phi_far + phi_self (and grad phi_far) by the five steps of Alg. 2 with the chosen split
    and window, float64."""
    x = np.mod(np.asarray(x, dtype=np.float64), vp.L)
    q = np.asarray(q, dtype=np.float64)
    m, P = vp.m, vp.P
    idx, w, dw = support(x, vp)
    a = np.zeros(m ** 3)                                       # step 1
    for jx in range(P):
        for jy in range(P):
            wxy = q * w[:, 0, jx] * w[:, 1, jy]
            base = (idx[:, 0, jx] * m + idx[:, 1, jy]) * m
            flat = (base[:, None] + idx[:, 2, :]).ravel()
            a += np.bincount(flat, weights=(wxy[:, None] * w[:, 2, :]).ravel(), minlength=m ** 3)
    ahat = np.fft.ifftn(a.reshape(m, m, m)) * m ** 3          # step 2 (e^{+})
    b = np.fft.fftn(scaling(vp) * ahat).real.reshape(-1)      # steps 3-4 (e^{-})
    n = x.shape[0]
    phi = np.zeros(n)
    g = np.zeros((n, 3)) if grad else None
    for jx in range(P):                                        # step 5
        for jy in range(P):
            base = (idx[:, 0, jx] * m + idx[:, 1, jy]) * m
            vals = b[base[:, None] + idx[:, 2, :]]
            sz = np.einsum("np,np->n", vals, w[:, 2, :])
            phi += w[:, 0, jx] * w[:, 1, jy] * sz
            if grad:
                dz = np.einsum("np,np->n", vals, dw[:, 2, :])
                g[:, 0] += dw[:, 0, jx] * w[:, 1, jy] * sz
                g[:, 1] += w[:, 0, jx] * dw[:, 1, jy] * sz
                g[:, 2] += w[:, 0, jx] * w[:, 1, jy] * dz
    phi -= self_coefficient(vp) * q
    return phi, g


def far_direct_variant(x, q, vp: VariantParams, K: int, grad: bool = False):
    """The split's Fourier series summed directly over 0 < |k| <= K (Alg. 1), plus the self
    term: the reference the comparisons measure errors against (``reference_modes`` gives a K
    whose neglected tail is far below the errors measured)."""
    x = np.mod(np.asarray(x, dtype=np.float64), vp.L)
    q = np.asarray(q, dtype=np.float64)
    L = vp.L
    a = np.arange(-K, K + 1)
    k2 = a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2
    keep = (k2 > 0) & (k2 <= K * K)
    kn = np.sqrt(np.arange(K * K + 1, dtype=np.float64))
    mt = np.zeros(kn.size)
    mt[1:] = mhat(2.0 * math.pi * kn[1:] / L, vp)
    B = np.where(keep, mt[np.minimum(k2, K * K)], 0.0) * structure_factor(x, q, L, K) / L ** 3
    ex, ey, ez = [t.conj() for t in _exp_tables(x, L, K)]
    t1 = np.einsum("abc,tc->tab", B, ez, optimize=True)
    t2 = np.einsum("tab,tb->ta", t1, ey)
    phi = np.einsum("ta,ta->t", t2, ex).real - self_coefficient(vp) * q
    g = None
    if grad:
        ik = -1j * 2.0 * math.pi / L * a
        g = np.zeros((x.shape[0], 3))
        g[:, 0] = np.einsum("ta,ta->t", t2 * ik[None, :], ex).real
        g[:, 1] = np.einsum("ta,ta->t", np.einsum("tab,tb->ta", t1, ey * ik[None, :]), ex).real
        t1z = np.einsum("abc,tc->tab", B * ik[None, None, :], ez, optimize=True)
        g[:, 2] = np.einsum("ta,ta->t", np.einsum("tab,tb->ta", t1z, ey), ex).real
    return phi, g


def reference_modes(vp: VariantParams, tail: float = 1e-16) -> int:
    """K for ``far_direct_variant``: for the PSWF split 4.7 times the band edge (as route R1 of
    ``direct``: the split's out-of-band tail decays slowly); for the Gaussian split the |k| at
    which exp(-sigma^2 w^2 / 4) falls below `tail`."""
    if vp.split == "pswf":
        return int(math.ceil(4.7 * vp.cs * vp.L / (2.0 * math.pi * vp.rc)))
    w = 2.0 * math.sqrt(math.log(1.0 / tail)) / vp.sigma
    return int(math.ceil(w * vp.L / (2.0 * math.pi)))
