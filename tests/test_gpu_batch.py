"""The batched engine (lbm_batch_*): every domain of an uneven batch must equal the
same lattice run alone (bitwise: same per-tile arithmetic) and the oracle, in the
per-step mode (one launch per step or per two steps) and in the persistent mode (one
launch for all pairs of steps of a call, per-domain barriers inside it).

The persistent kernel's scheduling protocol and the shape of its compiled loops are
checked on the CPU first (tests/test_persistent_protocol.py): an earlier form of its
barrier wait, a loop run by thread 0 alone, never finished on the GPU.  Every case
here prints its name before it runs."""
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


@pytest.mark.parametrize("mode", ["per_step", "per_step2", "persistent"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_lattices(lbm, mode, precision):
    say(f"batch {mode} {precision}")
    cfgs = _cfgs(precision)
    b = lbm.Batch(cfgs)
    if mode == "per_step2":  # two fused steps per launch; 7 and 30 steps end on single steps
        b.set_launch("per_step", 128, 16, steps_per_pass=2)
        assert b.launch["steps_per_pass"] == 2
    elif mode == "persistent":  # one launch of 3 (then 15) pairs, then one single step
        b.set_launch("persistent", 128, 16)
        assert b.launch["mode"] == "persistent" and b.launch["steps_per_pass"] == 2
    else:
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
    say("batch per-step vs oracle")
    cfgs = _cfgs("fp64")
    b = lbm.Batch(cfgs)
    b.set_launch("per_step", 64, 8)
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
    """Spin limit 0 (forced from the host): a tile that finds its domain's previous pair
    unfinished gives up at once, sets the error flag and every workgroup leaves; the
    launch ends and the host sees LBM_EDEVICE.  The batch runs again after a re-plan."""
    say("batch persistent: forced barrier timeout (spin limit 0)")
    cfgs = _cfgs("fp32")
    b = lbm.Batch(cfgs)
    b.set_launch("persistent", 128, 4, spin_limit=0, force_spin_limit=True)
    for i, d in enumerate(DOMAINS):
        b.init_field(i, _rho0(i, d))
    b.step(50)
    with pytest.raises(lbm.LBMError) as ei:
        b.sync()
    assert ei.value.status == -3
    b.set_launch("per_step", 64, 16)
    b.step(2)
    b.sync()


def test_batch_rejects_mixed_eos(lbm):
    say("batch mixed eos")
    with pytest.raises(lbm.LBMError):
        lbm.Batch([dict(nx=16, ny=16, eos="cs"), dict(nx=16, ny=16, eos="vdw", K=0.3, T_over_Tc=0.9)])


@pytest.mark.parametrize("tile", [(128, 16), (256, 8), (256, 16), (256, 24)])
def test_persistent_many_domains_equals_per_step(lbm, tile):
    """48 uneven domains (several per XCD group), three calls (1, 99 and 200 steps: a
    single step alone, 49 pairs and a single step, 100 pairs): the persistent engine is
    bitwise equal to per-step launches of the same tiles."""
    say(f"batch persistent, 48 domains, tile {tile}")
    rng = np.random.default_rng(5)
    e = th.carnahan_starling()
    _, Tc = th.critical_point(e)
    cfgs, rhos = [], []
    for i in range(48):
        nx, ny = int(rng.integers(12, 160)), int(rng.integers(12, 160))
        T = float(rng.uniform(0.7, 0.85))
        rv, rl = th.maxwell(e, T * Tc)
        cfgs.append(dict(nx=nx, ny=ny, eos="cs", precision="fp32", T_over_Tc=T,
                         A=float(rng.uniform(-0.7, -0.3)), kappa=float(rng.uniform(0.0, 0.8))))
        R = max(1.0, 0.3 * min(nx, ny))
        rhos.append(inputs.droplet(nx, ny, R, rl, rv, W=4.0, noise=1e-2, seed=100 + i))
    runs = {}
    for mode in ("persistent", "per_step"):
        b = lbm.Batch(cfgs)
        b.set_launch(mode, *tile, steps_per_pass=2)
        for i, r in enumerate(rhos):
            b.init_field(i, r)
        for k in (1, 99, 200):
            b.step(k)
        b.sync()
        assert all(o["step"] == 300 for o in b.observables())
        runs[mode] = [b.f_soa(i) for i in range(len(cfgs))]
        b.close()
    for i in range(len(cfgs)):
        assert np.array_equal(runs["persistent"][i], runs["per_step"][i], equal_nan=True), i


def test_persistent_default_tile(lbm):
    """The persistent mode's default row block is 24 rows (per-step: 16)."""
    b = lbm.Batch([dict(nx=40, ny=30, eos="cs", precision="fp32")])
    b.set_launch("persistent")
    assert (b.launch["tile_x"], b.launch["tile_y"], b.launch["steps_per_pass"]) == (256, 24, 2)
    b.set_launch("per_step")
    assert (b.launch["tile_x"], b.launch["tile_y"], b.launch["steps_per_pass"]) == (256, 16, 2)
    b.close()


def test_persistent_mode_needs_two_steps_per_pass(lbm):
    """The persistent engine runs two-step tiles: one step per pass or 64-lane tiles are
    refused (LBM_EINVAL) and the batch keeps its plan and still runs."""
    say("batch persistent: refused launch shapes")
    b = lbm.Batch(_cfgs("fp32")[:2])
    for kw in (dict(tile_x=64, tile_y=16), dict(tile_x=128, tile_y=16, steps_per_pass=1)):
        with pytest.raises(lbm.LBMError) as ei:
            b.set_launch("persistent", **kw)
        assert ei.value.status == -1
    assert b.launch["mode"] == "per_step"
    for i, d in enumerate(DOMAINS[:2]):
        b.init_field(i, _rho0(i, d))
    b.step(3)
    b.sync()


def test_one_graph_per_call_replayed(lbm):
    """All the launches of one lbm_batch_step call form one HIP graph, cached and replayed
    for the next call with the same step count (here 500 launches, replayed twice, with
    read-backs between): the domains stay bitwise the lattices run alone."""
    say("batch: one graph of 1000 steps, replayed")
    cfgs = _cfgs("fp32")
    b = lbm.Batch(cfgs)
    for i, d in enumerate(DOMAINS):
        b.init_field(i, _rho0(i, d))
    for rep in range(3):
        b.step(1000)
        b.observables()
    for i, (c, d) in enumerate(zip(cfgs, DOMAINS)):
        lat = lbm.Lattice(c)
        lat.init_field(_rho0(i, d))
        lat.step(3000)
        assert np.array_equal(b.f_soa(i), lat.f_soa()), i


def test_full_size_uneven_batch_sampled_domains(lbm, oracle_mod):
    """The uneven batch at full size (256 droplets, sides 64-512, about 25 M cells, FP32) in
    the library's default batch launch (two steps per launch, 256 x 16 tiles, one graph
    per call), 201 steps (100 two-step launches and a single step).  The draws are the
    first 256 of the seeded stream that pass the feasibility screen (draws below the
    lowest temperature at which the method holds two phases for their A, Sec. 3.1.2, are
    redrawn), so no domain may fault; every domain keeps its mass, five sampled domains
    (the smallest, the largest and three drawn) are bitwise the same lattice run alone,
    and the smallest domain matches the FP64 oracle; then the same 201 steps in the
    persistent launch give every domain bitwise the per-step state.  Densities start from
    the oracle's Maxwell construction for each draw."""
    from paper_1412_7228_amd import laplace

    say("uneven batch: feasibility screen of the draw stream")
    draws, report = laplace.feasible_batch_draws(256, 3)
    say(f"  {report['redraws']} redraws: " + ", ".join(
        f"T/Tc {r['T_over_Tc']:.3f} A {r['A']:.3f} ({r['reason']})" for r in report["rejected"]))
    assert len(draws) == 256 and report["redraws"] > 0
    assert all(r["T_over_Tc"] < 0.72 for r in report["rejected"])
    say("uneven batch, 256 domains, 201 steps")
    e = th.carnahan_starling()
    _, Tc = th.critical_point(e)
    cfgs, rhos = [], []
    for d in draws:
        rv, rl = th.maxwell(e, d["T_over_Tc"] * Tc)
        cfgs.append(dict(nx=d["nx"], ny=d["ny"], eos="cs", T_over_Tc=d["T_over_Tc"], A=d["A"],
                         kappa=d["kappa"], precision="fp32"))
        rhos.append(inputs.droplet(d["nx"], d["ny"], d["R"], rl, rv, W=5.0, noise=1e-3, seed=d["seed"]))
    cells = sum(c["nx"] * c["ny"] for c in cfgs)
    assert 24_000_000 < cells < 26_000_000
    b = lbm.Batch(cfgs)
    launch = b.launch
    assert (launch["mode"], launch["tile_x"], launch["tile_y"], launch["steps_per_pass"]) == \
        ("per_step", 256, 16, 2)
    for i, r in enumerate(rhos):
        b.init_field(i, r)
    m0 = np.array([o["mass"] for o in b.observables()])
    steps = 201
    b.step(steps)
    obs = b.observables()
    assert all(o["step"] == steps for o in obs)
    ok = [i for i, o in enumerate(obs) if o["n_nonfinite"] == 0 and o["n_domain"] == 0]
    say(f"  {len(ok)} of 256 domains without a fault after {steps} steps; failed at (T/Tc, A) "
        f"{sorted((round(cfgs[i]['T_over_Tc'], 3), round(cfgs[i]['A'], 3)) for i in range(256) if i not in ok)}")
    assert len(ok) == 256
    m1 = np.array([obs[i]["mass"] for i in ok])
    assert np.abs(m1 / m0[ok] - 1).max() < 1e-6
    sides = [c["nx"] for c in cfgs]
    small, large = int(np.argmin(sides)), int(np.argmax(sides))
    picks = [small, large] + [int(i) for i in np.random.default_rng(11).choice(256, 3, replace=False)]
    for i in picks:
        say(f"  domain {i}: {cfgs[i]['nx']}^2 against the lattice run alone")
        lat = lbm.Lattice(cfgs[i])
        lat.init_field(rhos[i])
        lat.step(steps)
        assert np.array_equal(b.f_soa(i), lat.f_soa(), equal_nan=True), i
        lat.close()
    small = min(ok, key=lambda i: sides[i])
    say(f"  domain {small}: {cfgs[small]['nx']}^2 against the FP64 oracle")
    o = oracle_mod.Oracle({k: v for k, v in cfgs[small].items() if k != "precision"}, nthreads=8)
    o.init_field(rhos[small])
    o.run(steps)
    want = o.fields()["rho"]
    got = b.field(small, "rho")
    assert float(np.abs(got - want).max() / np.abs(want).max()) < 1e-5
    # the same batch in the persistent launch (its default 256 x 24 tiles, 100 pairs in one
    # launch and a single step): every domain bitwise the per-step result
    say("  persistent launch, all 256 domains against the per-step run")
    per_step = [b.f_soa(i) for i in range(256)]
    b.set_launch("persistent")
    assert (b.launch["mode"], b.launch["tile_y"]) == ("persistent", 24)
    for i, r in enumerate(rhos):
        b.init_field(i, r)
    b.step(steps)
    assert all(o["step"] == 2 * steps for o in b.observables())  # the batch's clock runs on
    differ = [i for i in range(256) if not np.array_equal(b.f_soa(i), per_step[i], equal_nan=True)]
    assert differ == [], differ
    b.close()


# (A, T/Tc, feasible): the oracle's exact discrete flat-interface balance (N = 64) has a
# positive gas density at the first three points and only negative ones at the last two
SCREEN_POINTS = [(-0.5, 0.80, True), (-0.5, 0.70, True), (-0.7, 0.60, True),
                 (-0.3, 0.65, False), (-0.3, 0.60, False)]


def test_feasibility_screen_agrees_with_the_flat_balance(lbm):
    """The product-code feasibility screen (a flat slab of the draw's parameters run on the
    batched engine) accepts exactly the points where the oracle's exact steady flat balance
    has a positive gas density (Sec. 3.1.2: A bounds the lowest temperature), and its
    slab densities are the balance's (rho_l within 0.5%, rho_v within 5%)."""
    from paper_1412_7228_amd import laplace

    say("feasibility screen against the discrete flat balance")
    e = th.carnahan_starling()
    _, Tc = th.critical_point(e)
    cases = [dict(T_over_Tc=T, A=A, kappa=0.3) for A, T, _ in SCREEN_POINTS]
    res = laplace.screen_flat(cases)
    for (A, T, feasible), r in zip(SCREEN_POINTS, res):
        _, rv, rl = th.discrete_flat_balance(e, T * Tc, A, N=laplace.SCREEN_SLAB[0])
        say(f"  A={A} T/Tc={T}: screen {r}, balance rho_v={rv:.6g} rho_l={rl:.6g}")
        assert (rv > 0) == feasible
        assert r["ok"] == feasible, (A, T, r)
        if feasible:
            assert abs(r["rho_l"] / rl - 1) < 5e-3 and abs(r["rho_v"] / rv - 1) < 0.05
