"""Oracle: direct Ewald sums in float64 (no FFT).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``far_direct``  - the truncated Fourier-space sum of eq. Fsum / Alg. 1:
      phi_far(x) = 1/V sum_{k != 0, |k| <= K} Mhat(k) rhohat(k) e^{-2 pi i k.x / L},
      rhohat(k) = sum_j rho_j e^{+2 pi i k.x_j / L},   Mhat(k) = L^2/(pi |k|^2) gammahat(2 pi |k|/L),
  and its gradient (Remark rem:force, applied to the Fourier series). The exponential of a
  sum is the product of per-dimension exponentials, so rhohat over the cube [-K, K]^3 is
  assembled with matrix products (a library primitive) and the ball |k| <= K is masked.
* ``local_direct`` - the real-space residual phi_local (Sec. 3.1.1) with the compactly
  supported residual R(r) = (1 - Phi_{r_c}(r)) / r (eq. R), R = 0 for r >= r_c
  (Remark rem:compactsupport); pairs by brute force under the minimum image (r_c < L/2).
* ``self_term``   - phi_self,i = -lim_{r->0} M(r) rho_i (Sec. 3.1); with M = Phi_{r_c}(r)/r
  (eq. M) the limit is 2 gamma_{r_c}(0) = 2/(r_c lambda_0).
* ``gauss_ewald`` - the classical Gaussian split of Example 1, converged to ~1e-14, used only
  as an independent pin of the total potential.
* ``longrange_r1`` / ``longrange_r2`` - two routes to phi_far + phi_self for a given split:
  R1 sums the Fourier series directly up to K_ref; R2 takes the split-independent total
  potential from a tight split and subtracts the (exact, finite) real-space residual of the
  requested split.

Energy and forces follow the Remark in Sec. 3.1: E = 1/2 sum rho_i phi_i, F_i = -rho_i grad phi_i.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .pswf import PSWF, gammahat, split_function, split_function_deriv


def _mhat_table(Kmax2: int, L: float, rc: float, ps: PSWF) -> np.ndarray:
    """Mhat(k) as a function of the integer |k|^2 = 0..Kmax2 (entry 0 set to 0: neutrality)."""
    k2 = np.arange(Kmax2 + 1, dtype=np.float64)
    knorm = np.sqrt(k2)
    tab = np.zeros(Kmax2 + 1)
    nz = k2 > 0
    tab[nz] = L * L / (math.pi * k2[nz]) * gammahat(2.0 * math.pi * knorm[nz] / L, rc, ps)
    return tab


def _exp_tables(x: np.ndarray, L: float, K: int):
    """e^{2 pi i a x_d / L} for a = -K..K, one (n, 2K+1) table per dimension."""
    a = np.arange(-K, K + 1, dtype=np.float64)
    return [np.exp(1j * (2.0 * math.pi / L) * np.multiply.outer(x[:, d], a)) for d in range(3)]


def structure_factor(x: np.ndarray, q: np.ndarray, L: float, K: int, chunk: int = 65536) -> np.ndarray:
    """rhohat(k) = sum_j q_j e^{2 pi i k.x_j/L} on the cube k in [-K, K]^3 (index a + K)."""
    n = x.shape[0]
    W = 2 * K + 1
    rho = np.zeros((W, W, W), dtype=np.complex128)
    for s in range(0, n, chunk):
        ex, ey, ez = _exp_tables(x[s:s + chunk], L, K)
        qq = q[s:s + chunk]
        for a in range(W):
            A = (qq * ex[:, a])[:, None] * ey          # (nc, W) over b
            rho[a] += A.T @ ez                          # (W_b, W_c)
    return rho


def far_direct(x: np.ndarray, q: np.ndarray, L: float, rc: float, cs: float, K: int,
               targets: np.ndarray | None = None, grad: bool = True, chunk: int = 512):
    """Truncated Fourier-space sum (eq. Fsum) over 0 < |k| <= K at the target points.

    Returns (phi, grad_phi) with grad_phi None when grad is False.
    """
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    xt = x if targets is None else np.asarray(targets, dtype=np.float64)
    ps = PSWF(cs)
    V = L ** 3
    W = 2 * K + 1
    a = np.arange(-K, K + 1)
    k2 = a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2
    mask = (k2 <= K * K) & (k2 > 0)
    mtab = _mhat_table(K * K, L, rc, ps)
    Mk = np.where(mask, mtab[np.minimum(k2, K * K)], 0.0)
    B = Mk * structure_factor(x, q, L, K) / V           # 1/V Mhat(k) rhohat(k)
    two_pi_L = 2.0 * math.pi / L
    nt = xt.shape[0]
    phi = np.empty(nt)
    g = np.empty((nt, 3)) if grad else None
    Bz = B * (-1j * two_pi_L * a)[None, None, :]        # weight for d/dz
    for s in range(0, nt, chunk):
        ex, ey, ez = _exp_tables(xt[s:s + chunk], L, K)
        ex, ey, ez = ex.conj(), ey.conj(), ez.conj()    # e^{-2 pi i k.x/L}
        t1 = np.einsum("abc,tc->tab", B, ez, optimize=True)
        t2 = np.einsum("tab,tb->ta", t1, ey)
        phi[s:s + chunk] = np.einsum("ta,ta->t", t2, ex).real
        if grad:
            g[s:s + chunk, 0] = np.einsum("ta,ta->t", t2 * (-1j * two_pi_L * a)[None, :], ex).real
            t2y = np.einsum("tab,tb->ta", t1, ey * (-1j * two_pi_L * a)[None, :])
            g[s:s + chunk, 1] = np.einsum("ta,ta->t", t2y, ex).real
            t1z = np.einsum("abc,tc->tab", Bz, ez, optimize=True)
            t2z = np.einsum("tab,tb->ta", t1z, ey)
            g[s:s + chunk, 2] = np.einsum("ta,ta->t", t2z, ex).real
    return phi, g


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def local_direct(x: np.ndarray, q: np.ndarray, L: float, rc: float, cs: float,
                 target_idx: np.ndarray | None = None, grad: bool = True, chunk: int = 256):
    """phi_local,i = sum'_j rho_j R(|x_i - x_j|), R = (1 - Phi_{r_c})/r on r < r_c (eq. R).

    Targets are particles of the set (self pair excluded). Minimum image, so r_c < L/2.
    """
    if not rc < 0.5 * L:
        raise ValueError("local_direct needs r_c < L/2")
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    idx = np.arange(x.shape[0]) if target_idx is None else np.asarray(target_idx)
    ps = PSWF(cs)
    phi = np.zeros(idx.size)
    g = np.zeros((idx.size, 3)) if grad else None
    for s in range(0, idx.size, chunk):
        ti = idx[s:s + chunk]
        d = _min_image(x[ti][:, None, :] - x[None, :, :], L)      # (t, n, 3)
        r = np.sqrt(np.einsum("tnd,tnd->tn", d, d))
        near = (r < rc) & (ti[:, None] != np.arange(x.shape[0])[None, :])
        tt, jj = np.nonzero(near)
        rr = r[tt, jj]
        Phi = split_function(rr, rc, ps)
        R = (1.0 - Phi) / rr
        np.add.at(phi, tt + s, q[jj] * R)
        if grad:
            dR = -split_function_deriv(rr, rc, ps) / rr - (1.0 - Phi) / rr ** 2
            contrib = (q[jj] * dR / rr)[:, None] * d[tt, jj]
            np.add.at(g, tt + s, contrib)
    return phi, g


def self_term(q: np.ndarray, rc: float, cs: float) -> np.ndarray:
    """phi_self,i = -lim_{r->0} M(r) rho_i = -2 gamma_{r_c}(0) rho_i (Sec. 3.1, eq. M)."""
    ps = PSWF(cs)
    gamma0 = ps.psi(0.0) / (rc * ps.lambda0 * ps.psi_at_0)        # eq. PSWF_mollifier at 0
    return -2.0 * gamma0 * np.asarray(q, dtype=np.float64)


def k_ref_for(L: float, rc: float, cs: float, factor: float = 4.7) -> int:
    """Mode radius for route R1: the band edge K_max = c_s L / (2 pi r_c) times a factor so
    that the neglected tail (which decays like |k|^{-3/2} in RMS by Lemma 4 and Prop. 1) is
    an order of magnitude below the split error."""
    return int(math.ceil(factor * cs * L / (2.0 * math.pi * rc)))


def longrange_r1(x, q, L, rc, cs, K: int | None = None, targets=None, grad=True):
    """phi_far + phi_self at the particles by route R1 (direct Fourier sum up to K)."""
    K = k_ref_for(L, rc, cs) if K is None else K
    phi, g = far_direct(x, q, L, rc, cs, K, targets=targets, grad=grad)
    if targets is None:
        phi = phi + self_term(q, rc, cs)
    return phi, g


TIGHT_CS = 36.0


def longrange_r2(x, q, L, rc, cs, target_idx=None, grad=True, rc_o: float | None = None,
                 cs_o: float = TIGHT_CS):
    """phi_far + phi_self for split (rc, cs) at particle targets by route R2.

    The total periodic potential does not depend on the split (eq. potential2), so it is
    computed with a tight split (rc_o, cs_o; Fourier sum converged to ~1e-14) and the exact
    real-space residual of the requested split is subtracted:
        phi_far + phi_self = phi_total - phi_local^{(rc, cs)}.
    """
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    n = x.shape[0]
    idx = np.arange(n) if target_idx is None else np.asarray(target_idx)
    if rc_o is None:
        rc_o = 0.45 * L
    Ko = int(math.ceil(cs_o * L / (2.0 * math.pi * rc_o) * 1.02)) + 1
    far_o, gfar_o = far_direct(x, q, L, rc_o, cs_o, Ko, targets=x[idx], grad=grad)
    loc_o, gloc_o = local_direct(x, q, L, rc_o, cs_o, target_idx=idx, grad=grad)
    tot = far_o + loc_o + self_term(q[idx], rc_o, cs_o)
    loc, gloc = local_direct(x, q, L, rc, cs, target_idx=idx, grad=grad)
    phi = tot - loc + 0.0
    g = (gfar_o + gloc_o - gloc) if grad else None
    return phi, g


def total_potential(x, q, L, target_idx=None, grad=True, rc_o=None, cs_o=TIGHT_CS):
    """The full periodic Coulomb potential (eq. potential1, k = 0 dropped) via a tight split."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    idx = np.arange(x.shape[0]) if target_idx is None else np.asarray(target_idx)
    if rc_o is None:
        rc_o = 0.45 * L
    Ko = int(math.ceil(cs_o * L / (2.0 * math.pi * rc_o) * 1.02)) + 1
    far_o, gfar_o = far_direct(x, q, L, rc_o, cs_o, Ko, targets=x[idx], grad=grad)
    loc_o, gloc_o = local_direct(x, q, L, rc_o, cs_o, target_idx=idx, grad=grad)
    phi = far_o + loc_o + self_term(q[idx], rc_o, cs_o)
    return phi, ((gfar_o + gloc_o) if grad else None)


def gauss_ewald(x, q, L, sigma: float | None = None, K: int | None = None, images: int = 1,
                grad: bool = True):
    """Total potential with the classical Gaussian split (Example 1), converged to ~1e-14.

    phi_i = sum'_{j, r} rho_j erfc(|d|/sigma)/|d| + 1/V sum_{k != 0} 4 pi/w^2 e^{-sigma^2 w^2/4}
            Re[rhohat(k) e^{-i w.x_i}] - 2 rho_i / (sqrt(pi) sigma).
    """
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    n = x.shape[0]
    V = L ** 3
    if sigma is None:
        sigma = L / 12.0
    if K is None:
        K = int(math.ceil(2.0 * 6.2 / sigma * L / (2.0 * math.pi))) + 1
    phi = np.zeros(n)
    g = np.zeros((n, 3))
    rng = range(-images, images + 1)
    for rx in rng:
        for ry in rng:
            for rz in rng:
                shift = L * np.array([rx, ry, rz], dtype=np.float64)
                d = x[:, None, :] - x[None, :, :] + shift
                r = np.sqrt(np.einsum("ijd,ijd->ij", d, d))
                if rx == ry == rz == 0:
                    np.fill_diagonal(r, np.inf)
                phi += (erfc(r / sigma) / r) @ q
                dR = -2.0 / (math.sqrt(math.pi) * sigma) * np.exp(-(r / sigma) ** 2) / r - erfc(r / sigma) / r ** 2
                g += np.einsum("ij,ijd->id", dR / r * q[None, :], d)
    a = np.arange(-K, K + 1)
    k2 = a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2
    w2 = (2.0 * math.pi / L) ** 2 * np.maximum(k2, 1)
    Mk = np.where(k2 > 0, 4.0 * math.pi / w2 * np.exp(-sigma * sigma * w2 / 4.0), 0.0)
    B = Mk * structure_factor(x, q, L, K) / V
    ex, ey, ez = [t.conj() for t in _exp_tables(x, L, K)]
    two_pi_L = 2.0 * math.pi / L
    t1 = np.einsum("abc,tc->tab", B, ez, optimize=True)
    t2 = np.einsum("tab,tb->ta", t1, ey)
    phi += np.einsum("ta,ta->t", t2, ex).real
    if grad:
        g[:, 0] += np.einsum("ta,ta->t", t2 * (-1j * two_pi_L * a)[None, :], ex).real
        g[:, 1] += np.einsum("ta,ta->t", np.einsum("tab,tb->ta", t1, ey * (-1j * two_pi_L * a)[None, :]), ex).real
        t1z = np.einsum("abc,tc->tab", B * (-1j * two_pi_L * a)[None, None, :], ez, optimize=True)
        g[:, 2] += np.einsum("ta,ta->t", np.einsum("tab,tb->ta", t1z, ey), ex).real
    phi += -2.0 * q / (math.sqrt(math.pi) * sigma)
    return phi, (g if grad else None)


def energy(q, phi) -> float:
    """E = 1/2 sum_i rho_i phi_i (Remark in Sec. 3.1)."""
    return 0.5 * float(np.dot(np.asarray(q, dtype=np.float64), np.asarray(phi, dtype=np.float64)))


def forces(q, grad_phi) -> np.ndarray:
    """F_i = -rho_i grad phi_i (Remark in Sec. 3.1)."""
    return -np.asarray(q, dtype=np.float64)[:, None] * np.asarray(grad_phi, dtype=np.float64)
