"""The 200 x 200 Laplace sweep (Eq. 22; the droplet test of Sec. 3.1.1 and Sec. 4.1) at every
drop, FP32 and FP64 on the batched engine, against the FP64 oracle's observables stored in
tests/golden/laplace_sweep_200.json (written by tests/golden/make_laplace_sweep.py, which
calls only the oracle).

60 drops: R in {20, 30, 40, 50, 60}, T/Tc in {0.6, 0.7, 0.8}, kappa in {0, 0.3, 0.6} at
A = -0.5, and the A = -0.9 rows at 0.6 Tc; CS EOS, 20,000 steps, observed every 5,000.
Bars: after 20,000 steps, FP32 rho_l (centre), rho_v (corner) and sigma = dp R_e within 0.5%
of the oracle, FP64 every observable within 1e-9; each (A, T/Tc, kappa) group's Laplace fit
over the radii (the library's lbm_laplace_fit against the oracle's fit of the goldens)
within 0.5% in FP32.  At the earlier checkpoints the drops are still relaxing: dp (and with
it sigma) of a large drop passes through values far below its final one, where a relative
error measures the cancellation in p_in - p_out, not the path, so there each observable is
held to the same bar on its own scale, max(|value now|, |value after 20,000 steps|).  Each
observable's error is printed per drop and precision."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_1412_7228_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "laplace_sweep_200.json")
ERR_KEYS = ("mass", "rho_in", "rho_out", "dp", "R_e", "sigma", "max_u")


def say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device visible")
    from paper_1412_7228_amd import lbm as mod

    mod.load_library()
    return mod


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def initial_fields(golden):
    rhos = []
    for rec in golden["cases"]:
        c = rec["case"]
        rho = inputs.droplet(c["n"], c["n"], c["R"], rec["rho_l0"], rec["rho_v0"], W=c["W"],
                             noise=c["noise"], seed=c["seed"])
        digest = hashlib.sha256(np.ascontiguousarray(rho, dtype=np.float64).tobytes()).hexdigest()[:16]
        assert digest == rec["rho0_sha256_16"], c  # the oracle's input, bit for bit
        rhos.append(rho)
    return rhos


def run_batch(lbm, golden, rhos, precision):
    """All drops in one batch (the library's default batch launch); observables at every
    checkpoint of the goldens."""
    cfgs = [dict(nx=r["case"]["n"], ny=r["case"]["n"], eos="cs", T_over_Tc=r["case"]["T_over_Tc"],
                 A=r["case"]["A"], kappa=r["case"]["kappa"], precision=precision) for r in golden["cases"]]
    b = lbm.Batch(cfgs)
    for i, rho in enumerate(rhos):
        b.init_field(i, rho)
    out, done = {}, 0
    for s in golden["checkpoints"]:
        b.step(s - done)
        done = s
        out[str(s)] = b.observables(check=False)
    b.close()
    return out


def rel_err(g, o, scale=None):
    """|g - o| relative to max(|o|, |scale|)."""
    if o is None or not np.isfinite(g):
        return float("inf")
    den = max(abs(o), abs(scale) if scale is not None else 0.0)
    return abs(g - o) / den if den != 0 else abs(g)


def test_laplace_sweep_every_drop_against_the_oracle(lbm, golden):
    rhos = initial_fields(golden)
    say(f"laplace sweep: {len(rhos)} drops x {golden['checkpoints'][-1]} steps, fp32 and fp64 batches")
    gpu = {p: run_batch(lbm, golden, rhos, p) for p in ("fp32", "fp64")}
    fails = []
    worst = {p: {k: 0.0 for k in ERR_KEYS} for p in gpu}
    last = str(golden["checkpoints"][-1])
    for i, rec in enumerate(golden["cases"]):
        c = rec["case"]
        final = rec["observables"][last]
        for s in golden["checkpoints"]:
            orc = rec["observables"][str(s)]
            faulted = orc["n_nonfinite"] is None or orc["n_nonfinite"] > 0 or orc["n_domain"] > 0
            errs = {}
            for p in gpu:
                g = gpu[p][str(s)][i]
                g_fault = g["n_nonfinite"] > 0 or g["n_domain"] > 0
                if faulted or g_fault:
                    if faulted != g_fault:
                        fails.append((p, c, s, "fault status differs", g_fault, faulted))
                    continue
                errs[p] = {k: rel_err(g[k], orc[k], None if str(s) == last else final[k]) for k in ERR_KEYS}
                for k in ERR_KEYS:
                    worst[p][k] = max(worst[p][k], errs[p][k])
                bar = 5e-3 if p == "fp32" else 1e-9
                keys = ("rho_in", "rho_out", "sigma") if p == "fp32" else ERR_KEYS
                for k in keys:
                    if not errs[p][k] < bar:
                        fails.append((p, c, s, k, g[k], orc[k], errs[p][k]))
            if s == golden["checkpoints"][-1]:
                print("[observable-errors] " + json.dumps(dict(
                    A=c["A"], T_over_Tc=c["T_over_Tc"], kappa=c["kappa"], R=c["R"], steps=s,
                    **{p: {k: float(f"{v:.3e}") for k, v in e.items()} for p, e in errs.items()})), flush=True)
    print("[worst-observable-errors] " + json.dumps(
        {p: {k: float(f"{v:.3e}") for k, v in w.items()} for p, w in worst.items()}), flush=True)
    assert not fails, fails[:10]


def test_laplace_sweep_group_fits_against_the_oracle(lbm, golden):
    """Per (A, T/Tc, kappa): the Laplace fit of dp against 1/R_e over the five radii after
    20,000 steps, the library's lbm_laplace_fit on the FP32 batch against the oracle's fit
    of its own observables; and whether the group has relaxed (sigma of each drop moved by
    less than 1% over the last 5,000 steps in the oracle), printed."""
    import oracle

    rhos = initial_fields(golden)
    say("laplace sweep: group fits, fp32")
    last, prev = str(golden["checkpoints"][-1]), str(golden["checkpoints"][-2])
    gpu = run_batch(lbm, golden, rhos, "fp32")[last]
    groups = {}
    for i, rec in enumerate(golden["cases"]):
        c = rec["case"]
        groups.setdefault((c["A"], c["T_over_Tc"], c["kappa"]), []).append(i)
    fails = []
    for key, idx in sorted(groups.items()):
        orc = [golden["cases"][i]["observables"][last] for i in idx]
        s_orc, spread = oracle.laplace_fit([o["dp"] for o in orc], [o["R_e"] for o in orc])
        s_gpu, spread_gpu = lbm.laplace_fit([gpu[i]["dp"] for i in idx], [gpu[i]["R_e"] for i in idx])
        moved = [abs(golden["cases"][i]["observables"][last]["sigma"] /
                     golden["cases"][i]["observables"][prev]["sigma"] - 1) for i in idx]
        unrelaxed = [golden["cases"][i]["case"]["R"] for i, m in zip(idx, moved) if m > 0.01]
        print("[laplace-fit] " + json.dumps(dict(A=key[0], T_over_Tc=key[1], kappa=key[2], sigma_oracle=s_orc,
                                                 sigma_gpu_fp32=s_gpu, rel_err=abs(s_gpu / s_orc - 1),
                                                 spread_oracle=spread, spread_gpu=spread_gpu,
                                                 radii_not_relaxed=unrelaxed)), flush=True)
        if not abs(s_gpu / s_orc - 1) < 5e-3:
            fails.append((key, s_gpu, s_orc))
    assert not fails, fails
