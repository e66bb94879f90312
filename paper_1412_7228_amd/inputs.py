"""Seeded synthetic initial fields, shared by the GPU path's callers and the oracle's tests.

This module holds none of the lattice Boltzmann arithmetic: it only draws
random numbers and lays out initial density/velocity fields, so that both
sides of a parity check start from the same arrays.  Coexistence densities are
inputs here (the callers look them up), never computed.

Recipes (the workloads of the surface-tension study, Sec. 3.1.1, Sec. 3.1.2,
Sec. 4.1):

* ``droplet``  -- a circular drop of radius R at the lattice centre
  (nx/2, ny/2), tanh profile of width W between rho_l and rho_v, times
  (1 + noise * xi) with xi ~ U[-1, 1);
* ``slab``     -- a flat liquid layer (two straight interfaces), same profile;
* ``spinodal`` -- a uniform mean density times (1 + noise * xi);
* ``taylor_green`` -- the decaying Taylor-Green vortex velocity field;
* ``batch_draw_stream`` / ``batch_draws`` -- the uneven batch of Laplace
  droplets: integer side U{lo..hi}, R = u * side with u ~ U[r_lo, r_hi],
  T/Tc ~ U, kappa ~ U, A ~ U (the feasibility screen that redraws from the
  stream runs the method, so it lives with the runs, in ``laplace``).

All generators use numpy's PCG64 seeded with the given seed.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _noise(shape, noise: float, seed: int) -> np.ndarray:
    if noise == 0.0:
        return np.ones(shape)
    xi = rng(seed).uniform(-1.0, 1.0, size=shape)
    return 1.0 + noise * xi


def droplet(nx: int, ny: int, R: float, rho_l: float, rho_v: float, W: float = 5.0,
            noise: float = 1e-3, seed: int = 0, center=None) -> np.ndarray:
    """[ny, nx] density of a centred drop: (rl+rv)/2 - (rl-rv)/2 tanh(2(r-R)/W)."""
    cx, cy = (nx / 2.0, ny / 2.0) if center is None else center
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (r - R) / W)
    return rho * _noise(rho.shape, noise, seed)


def ellipse(nx: int, ny: int, Rx: float, Ry: float, rho_l: float, rho_v: float, W: float = 5.0,
            noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """[ny, nx] density of a centred elliptic drop with semi-axes Rx, Ry."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    dx, dy = x - nx / 2.0, y - ny / 2.0
    rr = np.sqrt((dx / Rx) ** 2 + (dy / Ry) ** 2)
    rmean = np.sqrt(Rx * Ry)
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (rr - 1.0) * rmean / W)
    return rho * _noise(rho.shape, noise, seed)


def slab(nx: int, ny: int, rho_l: float, rho_v: float, W: float = 5.0, noise: float = 0.0,
         seed: int = 0, axis: str = "x") -> np.ndarray:
    """[ny, nx] flat liquid layer occupying the middle half along ``axis``."""
    n = nx if axis == "x" else ny
    s = np.arange(n) + 0.5
    c1, c2 = n / 4.0, 3.0 * n / 4.0
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2 * (s - c1) / W) - np.tanh(2 * (s - c2) / W))
    rho = np.tile(prof, (ny, 1)) if axis == "x" else np.tile(prof[:, None], (1, nx))
    return rho * _noise(rho.shape, noise, seed)


def spinodal(nx: int, ny: int, rho_mean: float, noise: float = 1e-2, seed: int = 0) -> np.ndarray:
    """[ny, nx] uniform density rho_mean times (1 + noise * xi)."""
    return rho_mean * _noise((ny, nx), noise, seed)


def taylor_green(n: int, u0: float = 0.01, rho0: float = 1.0, modes: int = 1):
    """Density and velocity of the Taylor-Green vortex on an n x n periodic lattice at t = 0:
    ux = -u0 cos(kx) sin(ky), uy = u0 sin(kx) cos(ky), k = 2 pi modes / n."""
    k = 2.0 * np.pi * modes / n
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    return np.full((n, n), rho0), ux, uy


def batch_ranges() -> dict:
    """The uneven batch's draw ranges (workloads.json, ``uneven_batch_256``)."""
    from . import workloads

    w = workloads.get("uneven_batch_256")
    return dict(side=tuple(w["side"]), r_frac=tuple(w["r_frac"]), t_over_tc=tuple(w["T_over_Tc"]),
                kappa=tuple(w["kappa"]), A=tuple(w["A"]))


def batch_draw_stream(seed: int, side=None, r_frac=None, t_over_tc=None, kappa=None, A=None):
    """Endless seeded stream of independent draws of the uneven droplet batch, one dict per
    domain (``index`` counts the draws of the stream); a range left None is the
    workload's (:func:`batch_ranges`)."""
    d = batch_ranges()
    side = side or d["side"]
    r_frac = r_frac or d["r_frac"]
    t_over_tc = t_over_tc or d["t_over_tc"]
    kappa = kappa or d["kappa"]
    A = A or d["A"]
    g = rng(seed)
    i = 0
    while True:
        s = int(g.integers(side[0], side[1] + 1))
        yield dict(index=i, nx=s, ny=s,
                   R=float(g.uniform(*r_frac) * s),
                   T_over_Tc=float(g.uniform(*t_over_tc)),
                   kappa=float(g.uniform(*kappa)),
                   A=float(g.uniform(*A)),
                   seed=int(g.integers(0, 2**31 - 1)))
        i += 1


def batch_draws(n: int, seed: int, side=None, r_frac=None, t_over_tc=None, kappa=None,
                A=None) -> list[dict]:
    """The first n draws of :func:`batch_draw_stream` (no feasibility screen)."""
    stream = batch_draw_stream(seed, side, r_frac, t_over_tc, kappa, A)
    return [next(stream) for _ in range(n)]
