"""Laplace-law droplets (Eq. 22) in FP32 on the batched engine against the FP64
oracle: rho_l (centre), rho_v (corner) and sigma = dp R_e within 0.5 %, and the
Laplace fit over radii within 0.5 % of the oracle's fit.  200 x 200 lattice, CS EOS at 0.8Tc, A = -0.5,
kappa = 0.3, 20,000 steps.  Both sides start from the same droplets, built between the
oracle's Maxwell densities; each side fits the Laplace law with its own code (the
library's lbm_laplace_fit, the oracle's laplace_fit)."""
import os
import sys

import numpy as np
import pytest

from oracle import thermo as th
from paper_1412_7228_amd import inputs, laplace

pytestmark = pytest.mark.gpu


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


OBS_KEYS = ("mass", "rho_in", "rho_out", "dp", "R_e", "sigma", "max_u")


def test_fp32_laplace_droplets_match_fp64_oracle(lbm, oracle_mod):
    """Also reports each observable's relative error against the oracle, FP32 and FP64,
    and the density field's error for the R = 40 drop (printed as JSON lines)."""
    import json

    steps = 20000
    cases = [dict(n=200, R=R, T_over_Tc=0.8, A=-0.5, kappa=0.3, seed=i) for i, R in enumerate((20, 40, 60))]
    e = th.carnahan_starling()
    _, Tc = th.critical_point(e)
    rv, rl = th.maxwell(e, 0.8 * Tc)
    rhos = [inputs.droplet(200, 200, float(c["R"]), rl, rv, W=5.0, noise=1e-3, seed=c["seed"]) for c in cases]
    say(f"laplace fp32 + fp64 batches, 3 droplets x {steps} steps")
    gpu = laplace.run_cases(cases, steps, precision="fp32", rhos=rhos)
    gpu64 = laplace.run_cases(cases, steps, precision="fp64", rhos=rhos)
    assert all(r["ok"] for r in gpu) and all(r["ok"] for r in gpu64)
    nthr = int(os.environ.get("OMP_NUM_THREADS") or min(16, os.cpu_count() or 1))
    orc = []
    for c, g, g64, rho0 in zip(cases, gpu, gpu64, rhos):
        say(f"oracle R={c['R']}")
        cfg = dict(nx=200, ny=200, eos="cs", T_over_Tc=c["T_over_Tc"], A=c["A"], kappa=c["kappa"])
        o = oracle_mod.Oracle(cfg, nthreads=nthr)
        o.init_field(rho0)
        o.run(steps)
        ob = o.observables()
        orc.append(ob)
        err = {p: {k: abs(r[k] / ob[k] - 1) for k in OBS_KEYS} for p, r in (("fp32", g), ("fp64", g64))}
        if c["R"] == 40:
            ref = o.fields()["rho"]
            for p in ("fp32", "fp64"):
                lat = lbm.Lattice(dict(cfg, precision=p))
                lat.init_field(rho0)
                lat.step(steps)
                d = lat.field("rho") - ref
                err[p]["rho_field_linf"] = float(np.abs(d).max() / np.abs(ref).max())
                err[p]["rho_field_l2"] = float(np.sqrt((d * d).sum() / (ref * ref).sum()))
                lat.close()
        print("[observable-errors] " + json.dumps(dict(R=c["R"], steps=steps, **err)), flush=True)
        for k in ("rho_in", "rho_out", "sigma"):
            assert err["fp32"][k] < 5e-3, (c["R"], k, g[k], ob[k])
        for k in OBS_KEYS:
            assert err["fp64"][k] < 1e-9, (c["R"], k, g64[k], ob[k])
    # the Laplace fit over radii (finite-size effects of a drop of radius 60 in a
    # 200^2 periodic box are shared by both sides)
    s_gpu, _ = laplace.laplace_sigma(gpu)
    s_orc, spread = oracle_mod.laplace_fit([r["dp"] for r in orc], [r["R_e"] for r in orc])
    assert abs(s_gpu / s_orc - 1) < 5e-3 and spread < 0.1
