"""Throughput of the batched engine on the uneven droplet batch.

256 independent Laplace droplets, square domains with side uniform in
{64..512}, R = u * side with u ~ U[0.15, 0.35], T/Tc ~ U[0.6, 0.85],
kappa ~ U[0, 0.8], A ~ U[-0.7, -0.3] (seeded), FP32, CS EOS.  Times the
per-step launch mode (launches in HIP graphs) with one step per launch and
with two fused steps per launch, and the persistent mode (one launch for all
pairs of steps of a call), with HIP events on the batch's stream, and prints
one JSON line: MLUPS over all domains, the launch shapes, and how many
domains stayed two-phase.

Draws that the method cannot hold (laplace.feasible_batch_draws: a flat slab of
the draw's parameters faults, collapses or loses its second phase) are redrawn
from the same seeded stream, and the redraws are reported.

    python -m paper_1412_7228_amd.batchbench [--steps 20000] [--domains 256] [--no-screen]
        [--modes 1,2x128,2x256,p256] [--save-draws F | --load-draws F]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import autotune, inputs, laplace, lbm, runlog, workloads


def build(domains: int, seed: int, precision: str = "fp32", screen: bool = True,
          max_ratio: float | None = laplace.SCREEN_MAX_RATIO, draws_file: str | None = None):
    """The batch of `domains` droplets from the seeded draw stream: the first feasible
    draws (laplace.feasible_batch_draws, density-ratio cap `max_ratio`, None for none)
    unless screen is False, or the draws (and screen report) stored in `draws_file` by an
    earlier run.  Returns (batch, cases, cells, screen report)."""
    if draws_file:
        with open(draws_file) as fh:
            saved = json.load(fh)
        draws, report = saved["draws"], saved["report"]
    elif screen:
        draws, report = laplace.feasible_batch_draws(domains, seed, max_ratio=max_ratio)
    else:
        draws, report = inputs.batch_draws(domains, seed), None
    cases = [dict(n=d["nx"], R=d["R"], T_over_Tc=d["T_over_Tc"], A=d["A"], kappa=d["kappa"],
                  seed=d["seed"], screen_ratio=d.get("screen_ratio")) for d in draws]
    cfgs = [laplace.case_config(c, precision) for c in cases]
    b = lbm.Batch(cfgs)
    for i, (c, cfg) in enumerate(zip(cases, cfgs)):
        b.init_field(i, laplace.initial_density(c, cfg))
    cells = sum(c["n"] * c["n"] for c in cases)
    return b, cases, cells, report


def time_mode(b, mode, tile, steps, steps_per_pass=1):
    import torch

    b.set_launch(mode, *tile, steps_per_pass=steps_per_pass)
    b.step(10)
    b.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    b.sync()
    return e0.elapsed_time(e1)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    w = workloads.get("uneven_batch_256")
    ap.add_argument("--steps", type=int, default=w["steps"])
    ap.add_argument("--domains", type=int, default=w["domains"])
    ap.add_argument("--seed", type=int, default=w["seed"])
    ap.add_argument("--tune", action="store_true", help="run the autotuner first")
    ap.add_argument("--no-screen", action="store_true", help="keep infeasible draws (no redraw)")
    ap.add_argument("--max-ratio", type=float, default=laplace.SCREEN_MAX_RATIO,
                    help="screen: largest flat density ratio kept (0: no cap)")
    ap.add_argument("--modes", default="1,2x128,2x256,p256", help="launch modes to time")
    ap.add_argument("--log", default=None, help="append the result as one JSON line to this file (default: $LBM_RUN_LOG, unset = no log)")
    ap.add_argument("--save-draws", default=None, help="write the (screened) draws to this JSON file")
    ap.add_argument("--load-draws", default=None,
                    help="take the draws from a file written by --save-draws (no screen run; for profiling)")
    a = ap.parse_args()
    t0 = time.time()
    b, cases, cells, report = build(a.domains, a.seed, screen=not a.no_screen, max_ratio=a.max_ratio or None,
                                    draws_file=a.load_draws)
    if a.save_draws:
        with open(a.save_draws, "w") as fh:
            json.dump(dict(draws=[dict(nx=c["n"], ny=c["n"], R=c["R"], T_over_Tc=c["T_over_Tc"], A=c["A"],
                                       kappa=c["kappa"], seed=c["seed"], screen_ratio=c["screen_ratio"])
                                  for c in cases], report=report), fh)
    redraws = None if report is None else report["redraws"]
    print(f"[batch] {a.domains} domains, {cells} cells, {redraws} redraws, setup {time.time() - t0:.1f} s",
          flush=True)
    tuned = None
    if a.tune:
        tuned = autotune.tune_batch(b, steps=20, use_cache=False)
        print(f"[batch] autotune {tuned}", flush=True)
    res = {}
    all_modes = {"1": ("per_step", (64, 16), 1), "2x128": ("per_step", (128, 16), 2),
                 "2x256": ("per_step", (256, 16), 2), "p256": ("persistent", (256, 24), 2),
                 "p256x16": ("persistent", (256, 16), 2), "p128": ("persistent", (128, 16), 2)}
    for mode, tile, spp in (all_modes[m] for m in a.modes.split(",")):
        ms = time_mode(b, mode, tile, a.steps, spp)
        key = f"{mode}{'2' if spp == 2 and mode == 'per_step' else ''}_{tile[0]}x{tile[1]}"
        res[key] = dict(ms=ms, mlups=cells * a.steps / (ms * 1e-3) / 1e6, tile=list(tile),
                        steps_per_pass=spp, grid=b.launch["grid"], ntiles=b.launch["ntiles"])
        print(f"[batch] {key} {res[key]}", flush=True)
    obs = b.observables()
    ok = sum(1 for c, o in zip(cases, obs) if o["n_nonfinite"] == 0 and o["rho_in"] > 1.5 * o["rho_out"] > 0)
    faulted = [dict(domain=i, side=c["n"], R=round(c["R"], 2), T_over_Tc=round(c["T_over_Tc"], 4),
                    A=round(c["A"], 4), kappa=round(c["kappa"], 4), screen_ratio=c.get("screen_ratio"))
               for i, (c, o) in enumerate(zip(cases, obs)) if o["n_nonfinite"] > 0 or o["n_domain"] > 0]
    faults = len(faulted)
    line = dict(metric="MLUPS of the uneven droplet batch (FP32)", domains=a.domains, cells=cells,
                timed_steps_per_mode=a.steps, total_steps=len(res) * (a.steps + 10), modes=res,
                two_phase_domains=ok, domains_with_faults=faults, faulted=faulted,
                max_screen_ratio=max((c.get("screen_ratio") or 0) for c in cases),
                largest_screen_ratios=sorted(((c.get("screen_ratio") or 0) for c in cases), reverse=True)[:8],
                feasibility=None if report is None else dict(redraws=report["redraws"],
                                                             screen_steps=report["screen_steps"],
                                                             rejected=report["rejected"]),
                autotune=tuned, seconds=time.time() - t0)
    print(json.dumps(line), flush=True)
    runlog.append(dict(kind="batchbench", result=line), a.log)


if __name__ == "__main__":
    main()
