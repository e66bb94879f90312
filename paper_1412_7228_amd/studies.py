"""The paper's numerical studies, run on the GPU with the library's kernels.

Each study builds its seeded synthetic initial fields, runs them (many cases
at once on the batched engine, or single lattices where the field is sampled
in time) and returns a JSON-ready dict.  Nothing here computes lattice
Boltzmann arithmetic: initial densities come from the library's Maxwell
construction, everything after that from the GPU.

* ``laplace``     -- the CS Laplace sweep on 200 x 200 (R = 20..60, T/Tc in
  {0.6, 0.7, 0.8}, kappa in {0, 0.3, 0.6}, A = -0.5, plus A = -0.9 rows at
  0.6 Tc): sigma from the Laplace law (Eq. 22) per (T, kappa), and
  sigma(kappa)/sigma(0) against 1 - kappa (Eq. 28).
* ``asweep``      -- method 1 (Sec. 3.1): sigma of a R = 20 droplet on 100 x 100
  and the flat-interface densities for A from -0.9 to 0.99 (vdW, K = 0.3,
  0.9 Tc).
* ``kappa_sweep`` -- method 2 (Sec. 3.2.2): sigma of the same droplet and the
  flat-interface densities for kappa from 0 to 0.99 (vdW, K = 0.3, 0.9 Tc,
  A = -0.5), against the (1 - kappa) law of Eq. (28) and Table 1.
* ``stability``   -- the lowest temperature at which the model stays stable
  (Sec. 3.1.2 and Table 2) for A = -0.5 and 0.5 and every kappa of Table 2.
* ``pr_laplace``  -- the Peng-Robinson Laplace test of Sec. 4.1 (120 x 120,
  R = 20..40, kappa in {0, 0.9, 0.99}, 0.8 Tc, A = -0.3, K = 0.5).
* ``oscillation`` -- the elliptic-drop oscillation of Sec. 4.2 (Peng-Robinson
  as in Sec. 4.1, semi-axes 30 and 27, gas viscosity 0.2, liquid viscosity
  0.1 or 0.05, kappa in {-1, 0, 0.5}) against Eq. (30).

    python -m paper_1412_7228_amd.studies <name> [--out report.json]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs, laplace, lbm, oscillation, runlog

VDW_SEC3 = dict(eos="vdw", K=0.3)                  # Sec. 3: vdW with K = 0.3
PR_SEC4 = dict(eos="pr", K=0.5, T_over_Tc=0.8, A=-0.3)  # Sec. 4


def _finite(x):
    return float(x) if np.isfinite(x) else None


def _run_batch(cfgs, rhos, steps, tile=(128, 16), chunk=5000, steps_per_pass=2):
    b = lbm.Batch(cfgs)
    b.set_launch("per_step", *tile, steps_per_pass=steps_per_pass)
    for i, r in enumerate(rhos):
        b.init_field(i, r)
    left = steps
    while left > 0:
        k = min(chunk, left)
        b.step(k)
        left -= k
    obs = b.observables()
    b.close()
    return obs


def stable(o: dict, max_u: float = 0.1) -> bool:
    """A run counts as stable when its state is finite and positive, has no cell
    with U > 0, moves slower than max_u, and still holds two phases."""
    return bool(o["n_nonfinite"] == 0 and o["n_domain"] == 0 and o["rho_min"] > 0
                and np.isfinite(o["max_u"]) and o["max_u"] < max_u
                and o["rho_max"] > 1.5 * o["rho_min"])


# ---------------------------------------------------------------------------
def laplace_sweep(steps: int = 20000, precision: str = "fp32") -> dict:
    cases = laplace.full_sweep_cases()
    res = laplace.run_cases(cases, steps, precision=precision, tile=(128, 16))
    groups = {}
    for r in res:
        c = r["case"]
        groups.setdefault((c["A"], c["T_over_Tc"], c["kappa"]), []).append(r)
    rows = []
    for (A, T, k), rs in sorted(groups.items()):
        ok = [r for r in rs if r["ok"]]
        row = dict(A=A, T_over_Tc=T, kappa=k, runs=len(rs), two_phase=len(ok),
                   points=[dict(R=r["case"]["R"], R_e=r["R_e"], dp=r["dp"], rho_in=r["rho_in"],
                                rho_out=r["rho_out"], max_u=r["max_u"], ok=r["ok"]) for r in rs])
        if len(ok) >= 2:
            sig, spread = laplace.laplace_sigma(ok)
            row.update(sigma=sig, spread=spread, rho_l=float(np.mean([r["rho_in"] for r in ok])),
                       rho_v=float(np.mean([r["rho_out"] for r in ok])))
        else:
            row.update(sigma=None, note="outside the model's range: no two-phase steady state")
        rows.append(row)
    for row in rows:
        base = next((q for q in rows if q["A"] == row["A"] and q["T_over_Tc"] == row["T_over_Tc"]
                     and q["kappa"] == 0.0), None)
        if row.get("sigma") and base and base.get("sigma"):
            row["sigma_ratio"] = row["sigma"] / base["sigma"]
            row["one_minus_kappa"] = 1.0 - row["kappa"]
    return dict(study="laplace", lattice=200, steps=steps, precision=precision, rows=rows)


def a_sweep(As=None, steps: int = 20000, precision: str = "fp64") -> dict:
    As = list(np.round(np.concatenate([np.arange(-0.9, 0.95, 0.1), [0.95, 0.99]]), 4)) if As is None else As
    cfgs, rhos = [], []
    for A in As:
        cfg = dict(VDW_SEC3, nx=100, ny=100, T_over_Tc=0.9, A=float(A), kappa=0.0, precision=precision)
        rv, rl = lbm.coexistence(cfg)
        cfgs.append(cfg)
        rhos.append(inputs.droplet(100, 100, 20.0, rl, rv, W=5.0, noise=0.0))
        flat = dict(cfg, ny=4)
        cfgs.append(flat)
        rhos.append(inputs.slab(100, 4, rl, rv, W=5.0))
    obs = _run_batch(cfgs, rhos, steps, tile=(128, 16))
    rows = []
    for i, A in enumerate(As):
        d, f = obs[2 * i], obs[2 * i + 1]
        rows.append(dict(A=float(A), sigma=_finite(d["sigma"]) if stable(d) else None,
                         flat_rho_l=_finite(f["rho_max"]), flat_rho_v=_finite(f["rho_min"]),
                         droplet_stable=stable(d), flat_stable=stable(f)))
    lo = next(r for r in rows if abs(r["A"] - 0.99) < 1e-9)
    hi = next(r for r in rows if abs(r["A"] + 0.9) < 1e-9)
    shift = (hi["flat_rho_v"] / lo["flat_rho_v"] - 1.0) if lo["flat_rho_v"] and hi["flat_rho_v"] else None
    return dict(study="asweep", eos="vdw", K=0.3, T_over_Tc=0.9, steps=steps, precision=precision,
                rows=rows, gas_density_shift_A099_to_Am09=shift)


def kappa_sweep(kappas=(0.0, 0.2, 0.5, 0.7, 0.9, 0.99), steps: int = 20000,
                precision: str = "fp64") -> dict:
    """Method 2 (Sec. 3.2.2, Table 1, Fig. 3): for each kappa the R = 20 vdW droplet on
    100 x 100 (A = -0.5, 0.9 Tc, K = 0.3) and the flat interface, one batch: sigma by the
    Laplace law, sigma / sigma(kappa = 0) against 1 - kappa (Eq. 28), and the flat
    coexistence densities, which must not move with kappa (Table 1)."""
    cfgs, rhos = [], []
    for k in kappas:
        cfg = dict(VDW_SEC3, nx=100, ny=100, T_over_Tc=0.9, A=-0.5, kappa=float(k), precision=precision)
        rv, rl = lbm.coexistence(cfg)
        cfgs.append(cfg)
        rhos.append(inputs.droplet(100, 100, 20.0, rl, rv, W=5.0, noise=0.0))
        cfgs.append(dict(cfg, ny=4))
        rhos.append(inputs.slab(100, 4, rl, rv, W=5.0))
    obs = _run_batch(cfgs, rhos, steps, tile=(128, 16))
    rows = []
    s0 = obs[0]["sigma"] if stable(obs[0]) else None
    for i, k in enumerate(kappas):
        d, f = obs[2 * i], obs[2 * i + 1]
        sig = _finite(d["sigma"]) if stable(d) else None
        rows.append(dict(kappa=float(k), sigma=sig,
                         sigma_ratio=(sig / s0) if (sig and s0) else None,
                         linear_law=1.0 - float(k), flat_rho_l=_finite(f["rho_max"]),
                         flat_rho_v=_finite(f["rho_min"]), droplet_stable=stable(d), flat_stable=stable(f)))
    return dict(study="kappa_sweep", eos="vdw", K=0.3, T_over_Tc=0.9, A=-0.5, steps=steps,
                precision=precision, rows=rows)


def stability_scan(As=(-0.5, 0.5), kappas=(0.0, 0.2, 0.5, 0.7, 0.9, 0.99), temps=None,
                   geometry: str = "droplet", steps: int = 20000, precision: str = "fp64") -> dict:
    temps = list(np.round(np.arange(0.60, 0.905, 0.01), 3)) if temps is None else list(temps)
    cfgs, rhos, keys = [], [], []
    for A in As:
        for k in kappas:
            for T in temps:
                cfg = dict(VDW_SEC3, nx=100, ny=100, T_over_Tc=float(T), A=float(A), kappa=float(k),
                           precision=precision)
                rv, rl = lbm.coexistence(cfg)
                if geometry == "droplet":
                    r = inputs.droplet(100, 100, 20.0, rl, rv, W=5.0, noise=0.0)
                else:
                    r = inputs.slab(100, 100, rl, rv, W=5.0)
                cfgs.append(cfg)
                rhos.append(r)
                keys.append((A, k, T))
    obs = _run_batch(cfgs, rhos, steps, tile=(128, 16))
    table = {}
    for (A, k, T), o in zip(keys, obs):
        table.setdefault((A, k), []).append((T, stable(o), o))
    rows = []
    for (A, k), runs in sorted(table.items()):
        runs.sort(key=lambda t: t[0])
        t_min = None
        for T, ok, o in reversed(runs):  # lowest T with every higher T stable too
            if not ok:
                break
            t_min = (T, o)
        row = dict(A=A, kappa=k, T_min=None, ratio=None,
                   stable=[[T, ok] for T, ok, _ in runs])
        if t_min is not None:
            o = t_min[1]
            row.update(T_min=t_min[0], ratio=o["rho_max"] / o["rho_min"])
        rows.append(row)
    return dict(study="stability", geometry=geometry, eos="vdw", K=0.3, steps=steps,
                precision=precision, temps=temps, rows=rows)


def pr_laplace(kappas=(0.0, 0.9, 0.99), radii=(20, 25, 30, 35, 40), steps: int = 20000,
               precision: str = "fp64") -> dict:
    cases = [dict(n=120, R=R, kappa=k, seed=i, **PR_SEC4) for i, (k, R) in
             enumerate((k, R) for k in kappas for R in radii)]
    res = laplace.run_cases(cases, steps, precision=precision, tile=(128, 16))
    rows = []
    for k in kappas:
        rs = [r for r in res if r["case"]["kappa"] == k]
        ok = [r for r in rs if r["ok"]]
        row = dict(kappa=k, runs=len(rs), two_phase=len(ok),
                   points=[dict(R=r["case"]["R"], R_e=r["R_e"], dp=r["dp"], ok=r["ok"]) for r in rs])
        if len(ok) >= 2:
            sig, spread = laplace.laplace_sigma(ok)
            row.update(sigma=sig, spread=spread, rho_l=float(np.mean([r["rho_in"] for r in ok])),
                       rho_v=float(np.mean([r["rho_out"] for r in ok])))
        rows.append(row)
    s0 = rows[0].get("sigma")
    for row in rows:
        if s0 and row.get("sigma"):
            row["sigma_ratio"] = row["sigma"] / s0
            row["one_minus_kappa"] = 1.0 - row["kappa"]
    return dict(study="pr_laplace", lattice=120, steps=steps, precision=precision, **PR_SEC4, rows=rows)


def oscillation_study(kappas=(-1.0, 0.0, 0.5), nu_liquid=(0.1, 0.05), nu_gas: float = 0.2,
                      steps: int = 16000, precision: str = "fp64") -> dict:
    rows = []
    for k in kappas:
        for nl in nu_liquid:
            cfg = dict(PR_SEC4, nx=120, ny=120, kappa=k, precision=precision)
            rv, rl = lbm.coexistence(cfg)
            cfg.update(nu_gas=nu_gas, nu_liquid=nl, rho_gas=rv, rho_liquid=rl)
            try:
                r = oscillation.run(cfg, 30.0, 27.0, steps)
                rows.append(dict(kappa=k, nu_liquid=nl, period=r["period"], theory=r["theory"],
                                 error=r["error"], sigma=r["sigma"], rho_l=r["rho_l"],
                                 damping=r.get("damping")))
            except (RuntimeError, ValueError, lbm.LBMError) as ex:
                rows.append(dict(kappa=k, nu_liquid=nl, failed=str(ex)))
    return dict(study="oscillation", lattice=120, semi_axes=[30, 27], nu_gas=nu_gas, steps=steps,
                precision=precision, **PR_SEC4, rows=rows)


STUDIES = dict(laplace=laplace_sweep, asweep=a_sweep, kappa_sweep=kappa_sweep, stability=stability_scan,
               pr_laplace=pr_laplace, oscillation=oscillation_study)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("study", choices=sorted(STUDIES) + ["all"])
    ap.add_argument("--out", default=None, help="JSON report (default <study>.json)")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--log", default=None, help="append the result as one JSON line to this file (default: $LBM_RUN_LOG, unset = no log)")
    a = ap.parse_args()
    names = sorted(STUDIES) if a.study == "all" else [a.study]
    reports = {}
    for name in names:
        t0 = time.time()
        kw = {} if a.steps is None else dict(steps=a.steps)
        rep = STUDIES[name](**kw)
        rep["seconds"] = time.time() - t0
        reports[name] = rep
        print(f"[study] {name} done in {rep['seconds']:.1f} s", flush=True)
        runlog.append(dict(kind=f"study:{name}", result=rep), a.log)
    out = a.out or f"{a.study}.json"
    with open(out, "w") as f:
        json.dump(reports if a.study == "all" else reports[a.study], f, indent=1)
    print(json.dumps({k: v.get("seconds") for k, v in reports.items()}), flush=True)


if __name__ == "__main__":
    main()
