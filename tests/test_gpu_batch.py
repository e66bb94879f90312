"""The batched engine (lbm_batch_*): every domain of an uneven batch must equal the
same lattice run alone (bitwise: same per-tile arithmetic) in both launch modes, and
the oracle; a forced barrier timeout must end the launch with an error, not a hang."""
import sys

import numpy as np
import pytest

from oracle import thermo as th
from paper_1412_7228_amd import inputs

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


DOMAINS = [
    dict(nx=37, ny=23, T_over_Tc=0.7, A=-0.7, kappa=0.5, R=6),
    dict(nx=64, ny=64, T_over_Tc=0.8, A=-0.5, kappa=0.0, R=14),
    dict(nx=100, ny=70, T_over_Tc=0.75, A=-0.3, kappa=0.6, R=15),
    dict(nx=130, ny=130, T_over_Tc=0.85, A=-0.6, kappa=0.3, R=30),
    dict(nx=3, ny=5, T_over_Tc=0.8, A=-0.5, kappa=0.2, R=1),
]


def _cfgs(precision):
    out = []
    for d in DOMAINS:
        c = {k: v for k, v in d.items() if k != "R"}
        out.append(dict(c, eos="cs", precision=precision))
    return out


def _rho0(i, d):
    e = th.carnahan_starling()
    _, Tc = th.critical_point(e)
    rv, rl = th.maxwell(e, d["T_over_Tc"] * Tc)
    return inputs.droplet(d["nx"], d["ny"], d["R"], rl, rv, W=4.0, noise=1e-2, seed=i)


@pytest.mark.parametrize("mode", ["per_step", "persistent"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_lattices(lbm, mode, precision):
    say(f"batch {mode} {precision}")
    cfgs = _cfgs(precision)
    b = lbm.Batch(cfgs)
    b.set_launch(mode, 64, 16)
    for i, d in enumerate(DOMAINS):
        b.init_field(i, _rho0(i, d))
    b.step(7)
    b.step(30)
    b.sync()
    for i, (c, d) in enumerate(zip(cfgs, DOMAINS)):
        lat = lbm.Lattice(c)
        lat.init_field(_rho0(i, d))
        lat.step(37)
        assert np.array_equal(b.f_soa(i), lat.f_soa()), i


def test_batch_matches_oracle_fp64(lbm, oracle_mod):
    say("batch persistent vs oracle")
    cfgs = _cfgs("fp64")
    b = lbm.Batch(cfgs)
    b.set_launch("persistent", 64, 8)
    for i, d in enumerate(DOMAINS):
        b.init_field(i, _rho0(i, d))
    b.step(40)
    obs = b.observables()
    for i, (c, d) in enumerate(zip(cfgs, DOMAINS)):
        o = oracle_mod.Oracle(c, nthreads=4)
        o.init_field(_rho0(i, d))
        o.run(40)
        ref = o.f_soa()
        assert np.abs(b.f_soa(i) - ref).max() / np.abs(ref).max() < 1e-12, i
        ob = o.observables()
        assert abs(obs[i]["mass"] / ob["mass"] - 1) < 1e-12
        assert obs[i]["step"] == 40


def test_persistent_barrier_timeout_aborts_cleanly(lbm):
    """Spin limit 0: any tile that must wait gives up, sets the error flag and every
    workgroup leaves; the launch ends and the host sees LBM_EDEVICE."""
    say("batch forced barrier timeout")
    cfgs = _cfgs("fp32")
    b = lbm.Batch(cfgs)
    b.set_launch("persistent", 64, 4, spin_limit=0, force_spin_limit=True)
    for i, d in enumerate(DOMAINS):
        b.init_field(i, _rho0(i, d))
    b.step(50)
    with pytest.raises(lbm.LBMError) as ei:
        b.sync()
    assert ei.value.status == -3
    # the batch is usable again after a normal re-plan
    b.set_launch("per_step", 64, 16)
    b.step(2)
    b.sync()


def test_batch_rejects_mixed_eos(lbm):
    say("batch mixed eos")
    with pytest.raises(lbm.LBMError):
        lbm.Batch([dict(nx=16, ny=16, eos="cs"), dict(nx=16, ny=16, eos="vdw", K=0.3, T_over_Tc=0.9)])
