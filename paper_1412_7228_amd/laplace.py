"""Laplace-law droplet runs on the batched engine (Sec. 3.1.1 and Sec. 4.1, Eq. 22).

A droplet case is a dict with keys ``n`` (square lattice side), ``R`` (initial
radius), ``T_over_Tc``, ``A``, ``kappa`` and optionally ``seed``, ``W``
(interface width), ``eos`` and ``K``.  Cases run together in one
:class:`~paper_1412_7228_amd.lbm.Batch`; the result of a case is its FP64
observables: the inside/outside densities (rho_in at the centre, rho_out at
the corner), the pressure jump dp, the equimolar radius R_e and
sigma = dp * R_e.  Across radii, the Laplace fit of sigma is the
least-squares slope of dp against 1/R_e through the origin.

Everything numerical runs in the library's kernels; this module only builds
initial fields (tanh droplets between the Maxwell densities that the library
computes on the host) and collects results.

The uneven batch's parameter ranges reach temperatures below the lowest one at
which the model holds two phases for its A (Sec. 3.1.2: the gas branch
collapses).  :func:`feasible_batch_draws` screens every draw with the method
itself: its (T/Tc, A, kappa) run on a thin flat slab, the one-dimensional
coexistence problem of Table 1, and a draw that faults, collapses or loses its
second phase there is redrawn from the same seeded stream.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import inputs, lbm, workloads

_SWEEP = workloads.get("laplace_sweep_200")
_SCREEN = workloads.get("uneven_batch_256")["feasibility"]


def case_config(case: dict, precision: str = "fp32") -> dict:
    n = int(case["n"])
    cfg = dict(nx=n, ny=n, eos=case.get("eos", "cs"), T_over_Tc=float(case["T_over_Tc"]),
               A=float(case["A"]), kappa=float(case["kappa"]), precision=precision)
    if "K" in case:
        cfg["K"] = float(case["K"])
    return cfg


def initial_density(case: dict, cfg: dict) -> np.ndarray:
    rv, rl = lbm.coexistence(cfg)
    n = cfg["nx"]
    return inputs.droplet(n, n, float(case["R"]), rl, rv, W=float(case.get("W", 5.0)),
                          noise=float(case.get("noise", 1e-3)), seed=int(case.get("seed", 0)))


def run_cases(cases: list, steps: int, precision: str = "fp32", mode: str = "per_step",
              tile: tuple = (128, 16), chunk: int = 5000, steps_per_pass: int = 2,
              rhos: list | None = None) -> list:
    """Runs every case for `steps` steps in one batch; returns one result dict per case
    (the observables plus ``ok``: finite, positive densities, no U > 0 cell, a drop
    denser than its surroundings).  ``rhos``: initial densities, one per case (default:
    :func:`initial_density`)."""
    cfgs = [case_config(c, precision) for c in cases]
    b = lbm.Batch(cfgs)
    b.set_launch(mode, *tile, steps_per_pass=steps_per_pass)
    for i, (c, cfg) in enumerate(zip(cases, cfgs)):
        b.init_field(i, initial_density(c, cfg) if rhos is None else rhos[i])
    left = steps
    while left > 0:
        k = min(chunk, left)
        b.step(k)
        left -= k
    obs = b.observables()
    b.close()
    out = []
    for c, o in zip(cases, obs):
        ok = (o["n_nonfinite"] == 0 and o["n_domain"] == 0 and np.isfinite(o["sigma"])
              and o["rho_in"] > 1.5 * o["rho_out"] > 0 and o["dp"] > 0)
        out.append(dict(case=c, ok=bool(ok), **o))
    return out


def laplace_sigma(results: list) -> tuple[float, float]:
    """The library's Laplace fit (lbm_laplace_fit) of the results' dp and R_e: sigma
    through the origin of dp = sigma / R_e, and the relative spread of dp * R_e."""
    return lbm.laplace_fit([r["dp"] for r in results], [r["R_e"] for r in results])


def sweep_cases(radii=tuple(_SWEEP["radii"]), temps=tuple(_SWEEP["T_over_Tc"]),
                kappas=tuple(_SWEEP["kappa"]), A: float = _SWEEP["A"], n: int = _SWEEP["lattice"][0],
                extra_A=None) -> list:
    """The Laplace sweep: one droplet per (R, T/Tc, kappa) on an n x n lattice; with
    ``extra_A`` = (A', temps') also the rows (A', T) for T in temps'."""
    cases = []
    for T in temps:
        for k in kappas:
            for R in radii:
                cases.append(dict(n=n, R=R, T_over_Tc=T, A=A, kappa=k, seed=len(cases)))
    if extra_A is not None:
        a2, t2 = extra_A
        for T in t2:
            for k in kappas:
                for R in radii:
                    cases.append(dict(n=n, R=R, T_over_Tc=T, A=a2, kappa=k, seed=len(cases)))
    return cases


def full_sweep_cases() -> list:
    """The whole Laplace sweep workload: the (R, T/Tc, kappa) grid at its A and the extra
    rows at the other A (60 drops on 200 x 200)."""
    extra = _SWEEP["extra_rows"]
    return sweep_cases(extra_A=(extra["A"], tuple(extra["T_over_Tc"])))


SCREEN_SLAB = tuple(_SCREEN["slab"])     # flat slab: 64 cells across two interfaces, 4 rows
SCREEN_STEPS = _SCREEN["steps"]
SCREEN_MIN_RATIO = _SCREEN["min_ratio"]  # rho_max / rho_min that still counts as two phases
# largest flat density ratio kept: draws whose gas sinks towards zero (ratios of 10^4
# and more after the screen) hold on the slab for a while but fault as droplets
SCREEN_MAX_RATIO = _SCREEN["max_ratio"]


def screen_flat(cases: list, steps: int = SCREEN_STEPS, precision: str = "fp32",
                max_ratio: float | None = None) -> list:
    """Runs each case's (T/Tc, A, kappa, EOS) on a thin periodic flat slab (a liquid layer
    between the library's Maxwell densities) on the batched engine for `steps` steps.
    Returns one dict per case: ``ok`` (finite, positive, no U > 0 cell, rho_max / rho_min
    >= SCREEN_MIN_RATIO, and at most max_ratio unless that is None), the slab's liquid and
    gas densities and their ratio, and the reason when not ok."""
    nx, ny = SCREEN_SLAB
    cfgs = []
    for c in cases:
        cfg = dict(nx=nx, ny=ny, eos=c.get("eos", "cs"), T_over_Tc=float(c["T_over_Tc"]),
                   A=float(c["A"]), kappa=float(c["kappa"]), precision=precision)
        if "K" in c:
            cfg["K"] = float(c["K"])
        cfgs.append(cfg)
    b = lbm.Batch(cfgs)
    b.set_launch("per_step", 128, 16, steps_per_pass=2)
    for i, cfg in enumerate(cfgs):
        rv, rl = lbm.coexistence(cfg)
        b.init_field(i, inputs.slab(nx, ny, rl, rv, W=5.0))
    b.step(steps)
    obs = b.observables()
    b.close()
    out = []
    for o in obs:
        lo, hi = o["rho_min"], o["rho_max"]
        reason = None
        if o["n_nonfinite"] > 0 or not (np.isfinite(lo) and np.isfinite(hi)):
            reason = "non-finite or non-positive density"
        elif o["n_domain"] > 0:
            reason = "U > 0"
        elif not lo > 0.0:
            reason = "gas density not positive"
        elif hi < SCREEN_MIN_RATIO * lo:
            reason = "one phase left"
        elif max_ratio is not None and hi > max_ratio * lo:
            reason = f"density ratio above {max_ratio:g}"
        out.append(dict(ok=reason is None, rho_l=hi, rho_v=lo, ratio=(hi / lo) if lo > 0 else None,
                        reason=reason))
    return out


def feasible_batch_draws(n: int, seed: int, steps: int = SCREEN_STEPS,
                         max_ratio: float | None = SCREEN_MAX_RATIO, **ranges) -> tuple:
    """The first n draws of the seeded stream (inputs.batch_draw_stream) that pass
    :func:`screen_flat` with a density ratio of at most max_ratio, in stream order; returns
    (draws, report) with the number of draws rejected before the n-th kept one and each
    rejected draw's parameters and reason.  Each kept draw carries its slab's ratio."""
    stream = inputs.batch_draw_stream(seed, **ranges)
    kept, rejected, screened = [], [], 0
    while len(kept) < n:
        need = n - len(kept)
        cand = list(itertools.islice(stream, max(16, need + need // 4)))
        screened += len(cand)
        for d, r in zip(cand, screen_flat(cand, steps, max_ratio=max_ratio)):
            if len(kept) == n:
                break
            if r["ok"]:
                kept.append(dict(d, screen_ratio=r["ratio"]))
            else:
                rejected.append(dict(index=d["index"], T_over_Tc=d["T_over_Tc"], A=d["A"],
                                     kappa=d["kappa"], ratio=r["ratio"], reason=r["reason"]))
    return kept, dict(kept=len(kept), redraws=len(rejected), rejected=rejected, screen_steps=steps,
                      screen_slab=list(SCREEN_SLAB), max_ratio=max_ratio, screened=screened)
