"""Seeded synthetic particle systems shaped like the paper's workloads.

This module only draws inputs (positions, charges, box sizes). It holds none of the Ewald
method's arithmetic and is shared by the tests, the benchmark and the oracle's callers.
The paper's own experiments use uniformly random positions and normally distributed charges
shifted to neutrality (Sec. 7.1); no public dataset is involved.

All generators return float64 NumPy arrays: positions (n, 3) in [0, L)^3 and charges (n,)
that sum to zero (up to rounding), plus the box side L.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 16591
AVOGADRO = 6.02214076e23


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def paper_default(n: int = 100, seed: int = SEED_BASE, L: float = 1.0):
    """Sec. 7.1 setup: n uniform points in [0, L)^3, N(0,1) charges shifted to neutrality."""
    g = _rng(seed)
    x = g.random((n, 3)) * L
    q = g.standard_normal(n)
    q -= q.mean()
    return x, q, L


def uniform_pm1(n: int, seed: int = SEED_BASE, L: float = 1.0):
    """n uniform points, charges +-1 in equal numbers (n even), shuffled."""
    if n % 2:
        raise ValueError("n must be even for equal +-1 counts")
    g = _rng(seed)
    x = g.random((n, 3)) * L
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    g.shuffle(q)
    return x, q, L


def uniform_u11(n: int, seed: int = SEED_BASE, L: float = 1.0):
    """n uniform points, charges U[-1, 1] minus their mean."""
    g = _rng(seed)
    x = g.random((n, 3)) * L
    q = g.uniform(-1.0, 1.0, n)
    q -= q.mean()
    return x, q, L


def _random_rotations(g, k: int) -> np.ndarray:
    """k rotation matrices, uniform on SO(3) (normalised Gaussian quaternions)."""
    qu = g.standard_normal((k, 4))
    qu /= np.linalg.norm(qu, axis=1, keepdims=True)
    w, x, y, z = qu.T
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def water_box(n_mol: int = 10000, seed: int = SEED_BASE + 1, density_g_cm3: float = 1.0,
              r_oh: float = 0.1, angle_deg: float = 109.47, q_o: float = -0.8476):
    """Rigid 3-site water: O uniform at the given density (L in nm), H at r_oh from O with
    the HOH angle, random orientation, charges O = q_o and H = -q_o/2. Sites O, H, H per molecule."""
    g = _rng(seed)
    mass_g = n_mol * 18.01528 / AVOGADRO
    L = (mass_g / density_g_cm3 * 1e21) ** (1.0 / 3.0)  # cm^3 -> nm^3
    O = g.random((n_mol, 3)) * L
    half = math.radians(angle_deg) / 2.0
    body = np.array([[math.sin(half), 0.0, math.cos(half)],
                     [-math.sin(half), 0.0, math.cos(half)]]) * r_oh
    R = _random_rotations(g, n_mol)
    H = O[:, None, :] + np.einsum("kij,hj->khi", R, body)
    x = np.concatenate([O[:, None, :], H], axis=1).reshape(-1, 3)
    x = np.mod(x, L)
    q = np.tile(np.array([q_o, -q_o / 2.0, -q_o / 2.0]), n_mol)
    return x, q, L


def clustered(n: int = 100000, n_centres: int = 64, std: float = 0.02, seed: int = SEED_BASE + 3,
              L: float = 1.0):
    """Gaussian clusters of std `std`*L around uniform centres; +-1 charges in equal numbers."""
    if n % 2:
        raise ValueError("n must be even")
    g = _rng(seed)
    centres = g.random((n_centres, 3)) * L
    pick = g.integers(0, n_centres, n)
    x = np.mod(centres[pick] + g.standard_normal((n, 3)) * std * L, L)
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    g.shuffle(q)
    return x, q, L


def ensemble(n_sys: int = 256, n_lo: int = 500, n_hi: int = 20000, L_lo: float = 0.5, L_hi: float = 2.0,
             seed: int = SEED_BASE + 4):
    """Independent neutral systems: n log-uniform in [n_lo, n_hi] (even), L uniform in [L_lo, L_hi],
    uniform positions, +-1 charges. Returns a list of (x, q, L)."""
    g = _rng(seed)
    out = []
    for _ in range(n_sys):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        n += n % 2
        L = float(g.uniform(L_lo, L_hi))
        x = g.random((n, 3)) * L
        q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
        g.shuffle(q)
        out.append((x, q, L))
    return out


def nacl_cell(a: float = 1.0):
    """Conventional rock-salt cell: 4 cations (+1) and 4 anions (-1) in a cube of side a."""
    na = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)
    cl = np.array([[.5, 0, 0], [0, .5, 0], [0, 0, .5], [.5, .5, .5]], dtype=np.float64)
    x = np.concatenate([na, cl]) * a
    q = np.concatenate([np.ones(4), -np.ones(4)])
    return x, q, a


# Named configurations (the paper-shaped workloads this project measures).
def config(name: str):
    if name == "plain_fp64_n1000":
        return uniform_pm1(1000, seed=SEED_BASE + 0)
    if name == "water_n30000":
        return water_box(10000, seed=SEED_BASE + 1)
    if name == "uniform_n1e6":
        return uniform_u11(1_000_000, seed=SEED_BASE + 2)
    if name == "clustered_n1e5":
        return clustered(100_000, seed=SEED_BASE + 3)
    raise KeyError(name)
