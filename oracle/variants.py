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
in a cuboid box [0, L) x [0, Ly) x [0, Lz) with m x my x mz grid points (Sec. 6.1, remark on cuboid
domains; h^6 becomes prod_d h_d^2, and the window has the same P and c_w in grid units along each
axis, alpha_d = P h_d / 2),
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
    cw_window: float = 0.0    # PSWF window bandlimit; 0: pi P / 2 (eq. cwP)
    Ly: float | None = None   # cuboid sides and grid sizes along y and z (None: the x values)
    Lz: float | None = None
    my: int | None = None
    mz: int | None = None

    @property
    def sides(self):
        return (self.L, self.Ly or self.L, self.Lz or self.L)

    @property
    def grids(self):
        return (self.m, self.my or self.m, self.mz or self.m)

    @property
    def hs(self):
        return tuple(Ld / md for Ld, md in zip(self.sides, self.grids))

    @property
    def h(self) -> float:
        return self.L / self.m

    @property
    def alpha(self) -> float:
        return self.P * self.h / 2.0

    @property
    def cw(self) -> float:
        return self.cw_window if self.cw_window > 0 else math.pi * self.P / 2.0

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


def window_values(d, vp: VariantParams, axis: int = 0):
    """Window along `axis` and its derivative at offsets d = x - h_d l (any shape)."""
    h = vp.hs[axis]
    alpha = vp.P * h / 2.0
    if vp.window == "pswf":
        pw = PSWF(vp.cw)
        s = d / alpha
        return window_1d(s, pw), window_1d_deriv(s, pw) / alpha
    if vp.window == "gauss":
        s = d / alpha
        return gauss_window(s, vp.cg), gauss_window_deriv(s, vp.cg) / alpha
    if vp.window == "bspline":
        u = d / h
        return bspline(u, vp.P), bspline_deriv(u, vp.P) / h
    raise ValueError(vp.window)


def window_hat(k, vp: VariantParams, axis: int = 0):
    """phihat_d at integer wave numbers k along `axis` (the deconvolution factor of that axis)."""
    L, m, h = vp.sides[axis], vp.grids[axis], vp.hs[axis]
    alpha = vp.P * h / 2.0
    omega = 2.0 * math.pi * np.asarray(k, dtype=np.float64) / L
    if vp.window == "pswf":
        return window_hat_1d(omega, alpha, PSWF(vp.cw))
    if vp.window == "gauss":
        return gauss_window_hat(omega, alpha, vp.cg)
    if vp.window == "bspline":
        return h * spme_factor(k, m, vp.P)
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
    """Largest |k| kept (cubes): the PSWF split's band edge c_s L / (2 pi r_c), or m/2 for the Gaussian split."""
    if vp.split == "pswf":
        return vp.cs * vp.L / (2.0 * math.pi * vp.rc)
    return vp.m / 2.0


def band_omega(vp: VariantParams) -> float:
    """Largest |w| kept: c_s / r_c for the PSWF split; pi / max_d h_d (the Nyquist frequency of the
    coarsest axis, m/2 modes on a cube) for the Gaussian split."""
    if vp.split == "pswf":
        return vp.cs / vp.rc
    return math.pi / max(vp.hs)


# ---------------------------------------------------------------------------------------
# Alg. 2 with a chosen split and window
# ---------------------------------------------------------------------------------------

def kvec(m: int) -> np.ndarray:
    i = np.arange(m)
    return np.where(i <= (m - 1) // 2, i, i - m)


def support(x, vp: VariantParams):
    """Per particle and dimension: the P grid indices (mod m_d) l = floor(x/h_d - P/2) + 1 + j
    and the window values and derivatives at x - h_d l."""
    n = x.shape[0]
    idx = np.empty((n, 3, vp.P), dtype=np.int64)
    w = np.empty((n, 3, vp.P))
    dw = np.empty((n, 3, vp.P))
    for d in range(3):
        h, m = vp.hs[d], vp.grids[d]
        start = np.floor(x[:, d] / h - vp.P / 2.0).astype(np.int64) + 1
        l = start[:, None] + np.arange(vp.P)[None, :]
        w[:, d], dw[:, d] = window_values(x[:, d][:, None] - h * l, vp, d)
        idx[:, d] = np.mod(l, m)
    return idx, w, dw


def scaling(vp: VariantParams) -> np.ndarray:
    """s_k on the (m, my, mz) FFT bins: prod_d h_d^2 Mhat(|w|) / (V prod_d phihat_d^2), zero outside
    the band and at k = 0. For cubes the band is the |k| ball of ``band_edge``."""
    mx, my, mz = vp.grids
    Lx, Ly, Lz = vp.sides
    ks = [kvec(mm) for mm in vp.grids]
    w2 = ((2 * math.pi * ks[0] / Lx) ** 2)[:, None, None] + ((2 * math.pi * ks[1] / Ly) ** 2)[None, :, None] \
        + ((2 * math.pi * ks[2] / Lz) ** 2)[None, None, :]
    pref = np.prod(np.square(vp.hs)) / (Lx * Ly * Lz)
    cube = vp.sides[1] == vp.L and vp.sides[2] == vp.L and vp.grids[1] == vp.m and vp.grids[2] == vp.m
    if cube:   # exactly the cube's |k| ball (the same test as before, in integers)
        k2 = ks[0][:, None, None] ** 2 + ks[1][None, :, None] ** 2 + ks[2][None, None, :] ** 2
        kb = band_edge(vp)
        keep = (k2 > 0) & (k2 <= kb * kb * (1.0 + 1e-12))
        kn = np.sqrt(np.arange(int(k2.max()) + 1, dtype=np.float64))
        mt = np.zeros(kn.size)
        mt[1:] = mhat(2.0 * math.pi * kn[1:] / vp.L, vp)
        M = mt[k2]
    else:
        wb = band_omega(vp)
        keep = (w2 > 0) & (w2 <= wb * wb * (1.0 + 1e-12))
        M = np.zeros(w2.shape)
        M[keep] = mhat(np.sqrt(w2[keep]), vp)
    ph = [window_hat(ks[d], vp, d) for d in range(3)]
    phihat = ph[0][:, None, None] * ph[1][None, :, None] * ph[2][None, None, :]
    s = np.where(keep, pref * M / phihat ** 2, 0.0)
    return s


def fast_variant(x, q, vp: VariantParams, grad: bool = True):
    """phi_far + phi_self (and grad phi_far) by the five steps of Alg. 2 with the chosen split
    and window, float64."""
    x = np.mod(np.asarray(x, dtype=np.float64), np.asarray(vp.sides))
    q = np.asarray(q, dtype=np.float64)
    mx, my, mz = vp.grids
    P = vp.P
    idx, w, dw = support(x, vp)
    a = np.zeros(mx * my * mz)                                 # step 1
    for jx in range(P):
        for jy in range(P):
            wxy = q * w[:, 0, jx] * w[:, 1, jy]
            base = (idx[:, 0, jx] * my + idx[:, 1, jy]) * mz
            flat = (base[:, None] + idx[:, 2, :]).ravel()
            a += np.bincount(flat, weights=(wxy[:, None] * w[:, 2, :]).ravel(), minlength=mx * my * mz)
    ahat = np.fft.ifftn(a.reshape(mx, my, mz)) * (mx * my * mz)  # step 2 (e^{+})
    b = np.fft.fftn(scaling(vp) * ahat).real.reshape(-1)        # steps 3-4 (e^{-})
    n = x.shape[0]
    phi = np.zeros(n)
    g = np.zeros((n, 3)) if grad else None
    for jx in range(P):                                        # step 5
        for jy in range(P):
            base = (idx[:, 0, jx] * my + idx[:, 1, jy]) * mz
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


def far_direct_variant(x, q, vp: VariantParams, K: int, grad: bool = False, chunk: int = 2048):
    """The split's Fourier series summed directly over 0 < |w| <= 2 pi K / L_min (Alg. 1), plus the
    self term: the reference the comparisons measure errors against (``reference_modes`` gives a
    K whose neglected tail is far below the errors measured). On a cube: 0 < |k| <= K."""
    x = np.mod(np.asarray(x, dtype=np.float64), np.asarray(vp.sides))
    q = np.asarray(q, dtype=np.float64)
    Ls = vp.sides
    wK = 2.0 * math.pi * K / min(Ls)
    Kd = [int(math.ceil(wK * Ld / (2.0 * math.pi) * (1.0 + 1e-12))) for Ld in Ls]
    ax = [np.arange(-k, k + 1) for k in Kd]
    wd = [2.0 * math.pi * a / Ld for a, Ld in zip(ax, Ls)]
    w2 = wd[0][:, None, None] ** 2 + wd[1][None, :, None] ** 2 + wd[2][None, None, :] ** 2
    keep = (w2 > 0) & (w2 <= wK * wK * (1.0 + 1e-12))
    M = np.zeros(w2.shape)
    M[keep] = mhat(np.sqrt(w2[keep]), vp)
    # rhohat(k) = sum_j q_j e^{+i w.x_j}, per-axis exponential tables, summed in chunks
    rho = np.zeros(w2.shape, dtype=np.complex128)
    for s0 in range(0, x.shape[0], chunk):
        e = [np.exp(1j * np.multiply.outer(x[s0:s0 + chunk, d], wd[d])) for d in range(3)]
        qq = q[s0:s0 + chunk]
        for ia in range(len(ax[0])):
            A = (qq * e[0][:, ia])[:, None] * e[1]
            rho[ia] += A.T @ e[2]
    B = M * rho / (Ls[0] * Ls[1] * Ls[2])
    ex, ey, ez = [np.exp(-1j * np.multiply.outer(x[:, d], wd[d])) for d in range(3)]
    t1 = np.einsum("abc,tc->tab", B, ez, optimize=True)
    t2 = np.einsum("tab,tb->ta", t1, ey)
    phi = np.einsum("ta,ta->t", t2, ex).real - self_coefficient(vp) * q
    g = None
    if grad:
        g = np.zeros((x.shape[0], 3))
        g[:, 0] = np.einsum("ta,ta->t", t2 * (-1j * wd[0])[None, :], ex).real
        g[:, 1] = np.einsum("ta,ta->t", np.einsum("tab,tb->ta", t1, ey * (-1j * wd[1])[None, :]), ex).real
        t1z = np.einsum("abc,tc->tab", B * (-1j * wd[2])[None, None, :], ez, optimize=True)
        g[:, 2] = np.einsum("ta,ta->t", np.einsum("tab,tb->ta", t1z, ey), ex).real
    return phi, g


def reference_modes(vp: VariantParams, tail: float = 1e-16) -> int:
    """K for ``far_direct_variant``: for the PSWF split 4.7 times the band edge (as route R1 of
    ``direct``: the split's out-of-band tail decays slowly); for the Gaussian split the |k| at
    which exp(-sigma^2 w^2 / 4) falls below `tail`."""
    Lmin = min(vp.sides)
    if vp.split == "pswf":
        return int(math.ceil(4.7 * vp.cs * Lmin / (2.0 * math.pi * vp.rc)))
    w = 2.0 * math.sqrt(math.log(1.0 / tail)) / vp.sigma
    return int(math.ceil(w * Lmin / (2.0 * math.pi)))


def box_params(eps: float, sides, rc: float, tol_mode: str = "rel", q_l2: float = 0.0, n: int = 0,
               m: int | None = None):
    """Parameters for a cuboid box (Sec. 6.1, remark on cuboid domains): the cube of side
    L_min = min(sides) with the same particle and charge densities (n and ||rho||^2 scaled by
    L_min^3 / V) is parameterised by Alg. 3 (oracle/params.py), giving r_c, c_s, P and
    h = L_min / m; each axis then takes the smallest even 2,3,5,7-smooth m_d with L_d / m_d <= h."""
    from . import params as oparams
    Lx, Ly, Lz = (float(v) for v in sides)
    Lmin = min(Lx, Ly, Lz)
    ratio = Lmin ** 3 / (Lx * Ly * Lz)
    kw = dict(rc=rc, tol_mode=tol_mode)
    if tol_mode == "abs":
        kw["q_l2"] = q_l2 * math.sqrt(ratio)
    if m is not None:
        kw["m"] = m
    p = oparams.choose(eps, Lmin, **kw)
    h = Lmin / p.m
    ms = [oparams.next_smooth_even(int(math.ceil(Ld / h - 1e-9))) for Ld in (Lx, Ly, Lz)]
    return VariantParams(Lx, p.rc, p.cs, ms[0], p.P, Ly=Ly, Lz=Lz, my=ms[1], mz=ms[2])


def oversample(p, sigma: float) -> VariantParams:
    """PSWF/PSWF on a grid oversampled by sigma (a reading: the paper names oversampling as future
    work). m' is the smallest even 2,3,5,7-smooth size >= sigma m; with sigma' = m' / (2 k_band),
    k_band = c_s L / (2 pi r_c) modes, the band edge's first alias lies 2 pi / h - c_s / r_c away,
    i.e. pi P (1 - 1/(2 sigma')) / alpha; that is taken as the window bandlimit c_w, and P as the
    smallest support whose c_w reaches the base's c_w = pi P / 2 (Alg. 3). `p` is an
    oracle/params.py parameter set for a cube."""
    from . import params as oparams
    m2 = oparams.next_smooth_even(int(math.ceil(sigma * p.m - 1e-9)))
    kband = p.cs * p.L / (2.0 * math.pi * p.rc)
    shrink = math.pi * (1.0 - 1.0 / (2.0 * max(1.0, m2 / (2.0 * kband))))
    P = max(3, int(math.ceil(p.cw / shrink - 1e-9)))
    return VariantParams(p.L, p.rc, p.cs, m2, P, cw_window=shrink * P)
