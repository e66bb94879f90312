"""Capillary oscillation of an elliptic drop (Sec. 4.2, Eq. 30).

A drop with semi-axes (Rx, Ry) relaxes towards a circle of radius
R0 = sqrt(Rx Ry) and oscillates in the n = 2 mode.  The period is read from
the second-moment anisotropy a(t) = (Ixx - Iyy)/(Ixx + Iyy) of the excess
density rho - rho_min by a least-squares fit of a damped cosine; the
theory is T = 2 pi sqrt(rho_l R0^3 / (n (n^2 - 1) sigma)) (Eq. 30, with the
2 pi outside the square root), with sigma from the Laplace law of a round
drop of the same area.  The lattice runs are the library's kernels; this
module samples the density field and fits.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize

from . import inputs, lbm


def anisotropy(rho: np.ndarray) -> float:
    ny, nx = rho.shape
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    w = rho - rho.min()
    s = w.sum()
    cx, cy = (w * x).sum() / s, (w * y).sum() / s
    ixx = (w * (x - cx) ** 2).sum()
    iyy = (w * (y - cy) ** 2).sum()
    return float((ixx - iyy) / (ixx + iyy))


def fit_period(t: np.ndarray, a: np.ndarray) -> dict:
    """Least-squares a(t) = c + A exp(-g t) cos(2 pi t / T + phi); the initial T from
    the first two zero crossings of a - mean."""
    t = np.asarray(t, float)
    a = np.asarray(a, float)
    am = a - a[len(a) // 2:].mean()
    zc = [t[i] - am[i] * (t[i + 1] - t[i]) / (am[i + 1] - am[i]) for i in range(len(am) - 1) if am[i] * am[i + 1] < 0]
    T0 = 2.0 * (zc[1] - zc[0]) if len(zc) >= 2 else (t[-1] - t[0]) / 2
    f = lambda tt, c, A, g, T, ph: c + A * np.exp(-g * tt) * np.cos(2 * np.pi * tt / T + ph)
    p0 = (a[-1], a[0] - a[-1], 1.0 / max(T0, 1.0), T0, 0.0)
    p, _ = optimize.curve_fit(f, t, a, p0=p0, maxfev=20000)
    return dict(period=float(abs(p[3])), damping=float(p[2]), amplitude=float(p[1]))


def theory_period(rho_l: float, sigma: float, R0: float, mode: int = 2) -> float:
    return 2.0 * math.pi * math.sqrt(rho_l * R0 ** 3 / (mode * (mode ** 2 - 1) * sigma))


def run(cfg: dict, Rx: float, Ry: float, steps: int, every: int = 40, W: float = 5.0,
        laplace_steps: int = 10000) -> dict:
    """Oscillation of one elliptic drop and the Laplace sigma of a round drop of
    the same area, both on the GPU; cfg as for lbm.Lattice (square lattice)."""
    n = cfg["nx"]
    rv, rl = lbm.coexistence(cfg)
    lat = lbm.Lattice(cfg)
    lat.init_field(inputs.ellipse(n, n, Rx, Ry, rl, rv, W=W))
    ts, aa = [], []
    for k in range(steps // every):
        lat.step(every)
        ts.append((k + 1) * every)
        aa.append(anisotropy(lat.field("rho")))
    fit = fit_period(np.array(ts), np.array(aa))
    R0 = math.sqrt(Rx * Ry)
    drop = lbm.Lattice(cfg)
    drop.init_field(inputs.droplet(n, n, R0, rl, rv, W=W, noise=0.0))
    drop.step(laplace_steps)
    ob = drop.observables(check=False)
    Tth = theory_period(ob["rho_in"], ob["sigma"], R0)
    return dict(fit, theory=Tth, error=fit["period"] / Tth - 1.0, sigma=ob["sigma"], rho_l=ob["rho_in"],
                t=ts, anisotropy=aa)
