"""Seeded synthetic input generators shared by the tests, the oracle driver and bench.py.

This module holds only initial density/velocity fields and workload recipes (plain
parameter values); it holds none of the method's arithmetic (no EOS, no collision, no
force).  Every field is analytic (the paper's workloads are analytic initial
conditions), and every random choice comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np


def planar_density(nx: int, ny: int, rho_v: float, rho_l: float, W: float = 10.0,
                   axis: int = 1) -> np.ndarray:
    """Diffuse planar liquid slab, Eq. PlanarIntDensity.

    Interfaces at 0.25 N and 0.75 N along ``axis`` (1 = y as in the paper, 0 = x), node
    coordinates are the 0-based indices.  Returns a float64 [ny][nx] array.
    """
    n = ny if axis == 1 else nx
    s = np.arange(n, dtype=np.float64)
    y1, y2 = 0.25 * n, 0.75 * n
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(4.6 * (s - y1) / W) - np.tanh(4.6 * (s - y2) / W))
    if axis == 1:
        return np.ascontiguousarray(np.repeat(prof[:, None], nx, axis=1))
    return np.ascontiguousarray(np.repeat(prof[None, :], ny, axis=0))


def droplet_density(nx: int, ny: int, rho_v: float, rho_l: float, R: float, W: float = 5.0,
                    cx: float | None = None, cy: float | None = None) -> np.ndarray:
    """Circular droplet with a tanh rim (same 4.6/W convention as the planar profile)."""
    cx = 0.5 * nx if cx is None else cx
    cy = 0.5 * ny if cy is None else cy
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return np.ascontiguousarray(rho_v + 0.5 * (rho_l - rho_v) * (1.0 - np.tanh(4.6 * (r - R) / W)))


def droplet_on_film(nx: int, ny: int, rho_v: float, rho_l: float, R: float, h: float,
                    gap: float, V: float, W: float = 5.0):
    """Droplet of radius R above a liquid film of height h on the bottom wall (Sec. IV).

    The droplet centre sits ``gap`` nodes above the film surface plus R; the droplet moves
    with (0, -V) weighted by its tanh indicator.  Returns (rho, ux, uy) float64 [ny][nx].
    """
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    cx, cy = 0.5 * nx, h + gap + R
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    drop = 0.5 * (1.0 - np.tanh(4.6 * (r - R) / W))
    film = 0.5 * (1.0 - np.tanh(4.6 * (y - h) / W))
    phi = np.clip(drop + film, 0.0, 1.0)
    rho = rho_v + (rho_l - rho_v) * phi
    ux = np.zeros_like(rho)
    uy = -V * drop
    return np.ascontiguousarray(rho), ux, np.ascontiguousarray(uy)


def uniform_density(nx: int, ny: int, rho: float) -> np.ndarray:
    return np.full((ny, nx), float(rho))


def shear_wave(nx: int, ny: int, rho0: float, amp: float, k: int = 1):
    """u_x = amp sin(2 pi k y / ny) on a uniform density (textbook decay test)."""
    y = np.arange(ny, dtype=np.float64)
    ux = amp * np.sin(2 * np.pi * k * y / ny)
    ux2 = np.repeat(ux[:, None], nx, axis=1)
    return np.full((ny, nx), float(rho0)), np.ascontiguousarray(ux2), np.zeros((ny, nx))


def random_field(nx: int, ny: int, mean: float, amp: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return mean * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(ny, nx)))


def batched_planar_recipe(n_lattices: int = 64, seed: int = 0, Tr_lo: float = 0.35,
                          Tr_hi: float = 0.95, L_lo: int = 32, L_hi: int = 512):
    """Uneven batch of 1-D-like planar lattices: lengths 4*U{L_lo..L_hi}, Tr ~ U(Tr_lo, Tr_hi)."""
    rng = np.random.default_rng(seed)
    lengths = 4 * rng.integers(L_lo, L_hi + 1, size=n_lattices)
    trs = rng.uniform(Tr_lo, Tr_hi, size=n_lattices)
    return [int(v) for v in lengths], [float(t) for t in trs]


# ---------------------------------------------------------------------------
# Workload recipes: parameter values only, shared by bench.py, the GPU tests and the
# script that writes the oracle's stored results (tests/golden/).
# ---------------------------------------------------------------------------
# Shaped Peng-Robinson (a = 2/49, b = 2/21, omega = 0.344) with the Smooth loop
# (alpha = 0.3), raised vapor slope k_vap = 4 and EOS scale 0.25; Tr is set per workload.
SHAPED_PR = dict(base=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, scale=0.25, shape=1, alpha=0.3, k_vap=4.0)

# Static droplet (Laplace workload): 512 x 512 periodic, Tr = 0.5, R = 80, tanh rim of width 20,
# MRT with every rate 1 except the shear rates (tau_nu = 0.7), Li forcing with sigma from eps.
STATIC_DROPLET_512 = dict(nx=512, ny=512, eos=dict(SHAPED_PR, Tr=0.5), tau=[1, 1, 1, 1, 1, 1, 1, 0.7, 0.7],
                          R=80, W=20, steps=50000)

# Droplet impact on a liquid film between walls: 2048 x 1024, Tr = 0.47 (density ratio 3.07e4),
# droplet R = 100 moving at V = 0.072 with its rim 4 nodes above a film of height 40 = 0.2 D,
# tanh rims of width 16; shear relaxation time tau_l = 0.644 (Re = V D / nu = 300), every other
# rate 1; ghost densities rho_l below the bottom wall and rho_v above the top wall.
DROP_IMPACT_2048 = dict(nx=2048, ny=1024, eos=dict(SHAPED_PR, Tr=0.47), tau_l=0.644, R=100, h=40, gap=4, V=0.072,
                        W=16, parity_steps=2000)


def drop_impact_tau(recipe: dict) -> list:
    """Relaxation times of the drop-impact workload in the moment order (shear pair last)."""
    return [1.0] * 7 + [recipe["tau_l"]] * 2


def static_droplet_fields(recipe: dict, rho_v: float, rho_l: float) -> np.ndarray:
    return droplet_density(recipe["nx"], recipe["ny"], rho_v, rho_l, R=recipe["R"], W=recipe["W"])


def drop_impact_fields(recipe: dict, rho_v: float, rho_l: float):
    return droplet_on_film(recipe["nx"], recipe["ny"], rho_v, rho_l, R=recipe["R"], h=recipe["h"],
                           gap=recipe["gap"], V=recipe["V"], W=recipe["W"])
