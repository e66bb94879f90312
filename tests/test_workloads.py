"""The workloads as data (paper_1412_7228_amd/workloads.json) and the run log
(paper_1412_7228_amd/runlog.py): every consumer takes the same numbers, the
stored Laplace-sweep goldens were written for exactly the sweep the data
describes, the seeded batch stream still starts where it did, and the log
writes one parseable JSON line per record."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1412_7228_amd import inputs, laplace, runlog, workloads  # noqa: E402


def test_workload_names():
    assert workloads.names() == ["droplet_100", "laplace_sweep_200", "lattice_4096_spinodal",
                                 "surrogate_sigma_targets", "uneven_batch_256"]
    with pytest.raises(KeyError):
        workloads.get("nope")


def test_bench_takes_its_workloads_from_the_data():
    import bench

    assert bench.N == 4096
    assert bench.WORKLOAD == dict(nx=4096, ny=4096, eos="cs", T_over_Tc=0.7, A=-0.5, kappa=0.0)
    assert bench.DROPLET_100 == dict(nx=100, ny=100, eos="cs", T_over_Tc=0.8, A=-0.5, kappa=0.0)
    assert (bench.DROP_R, bench.DROP_W, bench.DROP_NOISE, bench.DROP_SEED, bench.DROP_STEPS) == \
        (25.0, 5.0, 1e-3, 0, 5000)
    assert (bench.SPINODAL_NOISE, bench.SPINODAL_SEED) == (0.01, 0)


def test_spinodal_mean_density_is_the_mean_of_the_coexistence_densities():
    """rho_mean of the throughput lattice: (rho_v + rho_l) / 2 of CS at 0.7 Tc, from the
    oracle's Maxwell construction (to the 6 digits stored)."""
    import oracle

    e = oracle.thermo.carnahan_starling()
    _, Tc = oracle.thermo.critical_point(e)
    rv, rl = oracle.thermo.maxwell(e, 0.7 * Tc)
    assert abs(workloads.get("lattice_4096_spinodal")["rho_mean"] - (rv + rl) / 2) < 1e-6


def test_laplace_sweep_goldens_cover_exactly_the_sweep_workload():
    with open(os.path.join(ROOT, "tests", "golden", "laplace_sweep_200.json")) as fh:
        golden = json.load(fh)
    w = workloads.get("laplace_sweep_200")
    cases = laplace.full_sweep_cases()
    assert len(cases) == len(golden["cases"]) == 60
    for c, g in zip(cases, golden["cases"]):
        g = g["case"]
        assert (c["n"], float(c["R"]), c["T_over_Tc"], c["A"], c["kappa"], c["seed"]) == \
            (g["n"], g["R"], g["T_over_Tc"], g["A"], g["kappa"], g["seed"])
        assert (g["W"], g["noise"]) == (w["droplet"]["W"], w["droplet"]["noise"])
    assert golden["checkpoints"] == w["checkpoints"]


def test_batch_stream_head_is_unchanged():
    """The first draw of the uneven batch's seeded stream (seed 3), as the feasibility
    screen, the batch benchmark and the profiles saw it."""
    d = next(inputs.batch_draw_stream(workloads.get("uneven_batch_256")["seed"]))
    assert (d["nx"], d["ny"], d["seed"]) == (428, 428, 183930185)
    assert d["R"] == 84.47097936462613 and d["T_over_Tc"] == 0.8003186163015992
    assert d["kappa"] == 0.46572962885149427 and d["A"] == -0.6623485431038403
    r = inputs.batch_ranges()
    assert r == dict(side=(64, 512), r_frac=(0.15, 0.35), t_over_tc=(0.6, 0.85), kappa=(0.0, 0.8),
                     A=(-0.7, -0.3))
    assert (laplace.SCREEN_SLAB, laplace.SCREEN_STEPS, laplace.SCREEN_MAX_RATIO) == ((64, 4), 20000, 1000.0)


def test_surrogate_study_constants():
    from paper_1412_7228_amd import surrogate

    assert (surrogate.TOLERANCE, surrogate.VERIFY_N, surrogate.VERIFY_R, surrogate.VERIFY_STEPS) == \
        (0.02, 200, 40.0, 20000)
    assert workloads.get("surrogate_sigma_targets")["network"] == [3, 128, 128, 128, 3]


def test_run_log(tmp_path, monkeypatch):
    monkeypatch.delenv(runlog.ENV, raising=False)
    assert runlog.append({"kind": "x"}) is None  # no file configured: nothing written
    p = tmp_path / "runs.jsonl"
    assert runlog.append({"kind": "bench", "result": {"value": 1.5}}, str(p)) == str(p)
    monkeypatch.setenv(runlog.ENV, str(p))
    runlog.append({"kind": "batchbench", "result": {"value": 2}})
    lines = [json.loads(l) for l in p.read_text().splitlines()]
    assert [l["kind"] for l in lines] == ["bench", "batchbench"]
    for l in lines:
        assert {"time", "host", "argv", "library", "kind", "result"} <= set(l)
        assert l["host"]["cpus"] == os.cpu_count()


def test_batch_build_screens_with_the_ratio_cap_by_default():
    """batchbench.build (used by the batch benchmark and bench.py) screens the draw stream
    with the workload's density-ratio cap unless told otherwise."""
    import inspect

    from paper_1412_7228_amd import batchbench

    assert inspect.signature(batchbench.build).parameters["max_ratio"].default == laplace.SCREEN_MAX_RATIO == 1000.0
    assert inspect.signature(laplace.feasible_batch_draws).parameters["max_ratio"].default == 1000.0
