"""Oracle: parameter selection for the PSWF/PSWF method (Alg. 3, Sec. 6).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Steps, in the paper's order (Alg. 3):
  1. c_s = 1/2 W_0(2 (B_s/eps)^2), B_s = A_s ||rho||_2 sqrt(r_c) / sqrt(V)   (eq. cs_dimless)
     or, in the relative-tolerance mode, c_s = log(1/eps)                     (Sec. 6.2.1)
  2. c_w = -1/2 W(-2 B_w^2 e^{-2 c_s} / c_s), B_w = (A_s/A_w) sqrt(r_c/L)       (eq. cwW)
  3. alpha = r_c c_w / c_s                                                    (eq. alpha)
  4. m = ceil(L c_s / (pi r_c))                                               (eq. m_cs_dimless)
  5. P = ceil(2 alpha m / L)                                                  (eq. P_dimless)

Readings where the paper is silent (each listed in the design notes):
  * the Lambert-W branch in step 2 is W_{-1}: W_0 of the tiny negative argument gives
    c_w ~ 0, while the balance equation eq. cwcs_model_dimless needs c_w > 1/2;
  * step 4 is followed by rounding m up to an even size whose prime factors are 2, 3, 5, 7
    (the paper assumes even m in Sec. 6); step 5 uses that final m;
  * the method then runs with c_s = pi r_c m / L, c_w = pi P / 2 and alpha = P h / 2, the
    relations of eq. csrc, eq. cwP and Sec. 6.3 that the paper's experiments use;
  * A_s = 5 (Sec. 5.1.1) and A_s/A_w = 4 sqrt(5) / pi^{3/2} (Sec. 6.3);
  * when the grid size m is prescribed instead of r_c, r_c is solved from eq. csrc;
  * with neither given, r_c keeps a mean of 64 neighbours: r_c = L (3*64/(4 pi n))^{1/3}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import lambertw

A_S = 5.0
A_S_OVER_A_W = 4.0 * math.sqrt(5.0) / math.pi ** 1.5
DEFAULT_NEIGHBOURS = 64.0


@dataclass
class Params:
    L: float
    eps: float
    tol_mode: str  # "rel" or "abs"
    rc: float
    cs: float
    cw: float
    alpha: float
    m: int
    P: int
    # unrounded values of steps 1-3, for reference
    cs_alg: float
    cw_alg: float
    alpha_alg: float

    @property
    def h(self) -> float:
        return self.L / self.m


def is_smooth_even(m: int) -> bool:
    if m < 2 or m % 2:
        return False
    for p in (2, 3, 5, 7):
        while m % p == 0:
            m //= p
    return m == 1


def next_smooth_even(m: int) -> int:
    m = max(int(m), 2)
    while not is_smooth_even(m):
        m += 1
    return m


def cs_from_eps(eps: float, L: float, rc: float, q_l2: float, tol_mode: str) -> float:
    if tol_mode == "rel":
        return math.log(1.0 / eps)
    Bs = A_S * q_l2 * math.sqrt(rc) / math.sqrt(L ** 3)
    return 0.5 * float(lambertw(2.0 * (Bs / eps) ** 2, 0).real)


def cw_from_cs(cs: float, rc: float, L: float) -> float:
    Bw = A_S_OVER_A_W * math.sqrt(rc / L)
    arg = -2.0 * Bw * Bw * math.exp(-2.0 * cs) / cs
    if not (-1.0 / math.e < arg < 0.0):
        raise ValueError("no real W_{-1} solution for c_w")
    return -0.5 * float(lambertw(arg, -1).real)


def choose(eps: float, L: float, *, rc: float | None = None, m: int | None = None,
           n: int | None = None, q_l2: float | None = None, tol_mode: str = "rel") -> Params:
    if tol_mode not in ("rel", "abs"):
        raise ValueError("tol_mode")
    if tol_mode == "abs" and q_l2 is None:
        raise ValueError("abs mode needs ||rho||_2")
    q = 0.0 if q_l2 is None else float(q_l2)
    if rc is None and m is None:
        if n is None:
            raise ValueError("need rc, m or n")
        rc = L * (3.0 * DEFAULT_NEIGHBOURS / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    if rc is None:
        # grid prescribed: solve eq. csrc for r_c (c_s depends on r_c only in abs mode)
        if not is_smooth_even(m):
            raise ValueError("prescribed m must be even with factors 2,3,5,7")
        rc = L * math.log(1.0 / eps) / (math.pi * m)
        for _ in range(200):
            rc_new = L * cs_from_eps(eps, L, rc, q, tol_mode) / (math.pi * m)
            if abs(rc_new - rc) <= 1e-15 * rc:
                rc = rc_new
                break
            rc = rc_new
    cs = cs_from_eps(eps, L, rc, q, tol_mode)          # step 1
    cw = cw_from_cs(cs, rc, L)                          # step 2
    alpha = rc * cw / cs                                # step 3
    m_raw = L * cs / (math.pi * rc)                     # step 4
    m_alg = int(math.ceil(m_raw - 1e-9))
    m_fin = next_smooth_even(m_alg) if m is None else int(m)
    if m is not None and m_alg > m_fin:
        raise ValueError("prescribed m too small")
    P = int(math.ceil(2.0 * alpha * m_fin / L - 1e-9))  # step 5
    h = L / m_fin
    return Params(L=float(L), eps=float(eps), tol_mode=tol_mode, rc=float(rc),
                  cs=math.pi * rc * m_fin / L, cw=math.pi * P / 2.0, alpha=P * h / 2.0,
                  m=m_fin, P=P, cs_alg=cs, cw_alg=cw, alpha_alg=alpha)


def split_error_model(p: Params, q_l2: float) -> float:
    """eq. PSWF_model: A_s ||rho|| / sqrt(V) * sqrt(r_c) c_s^{-1/2} e^{-c_s}."""
    return A_S * q_l2 / math.sqrt(p.L ** 3) * math.sqrt(p.rc) * p.cs ** -0.5 * math.exp(-p.cs)


def window_error_model(p: Params, q_l2: float) -> float:
    """eq. window_err_model: A_w ||rho|| / sqrt(V) * sqrt(L) c_w^{1/2} e^{-c_w}."""
    A_w = A_S / A_S_OVER_A_W
    return A_w * q_l2 / math.sqrt(p.L ** 3) * math.sqrt(p.L) * p.cw ** 0.5 * math.exp(-p.cw)


def smooth_sizes(lo: int, hi: int) -> np.ndarray:
    return np.array([k for k in range(lo, hi + 1) if is_smooth_even(k)])
