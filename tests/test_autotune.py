"""The autotuner's cache keys and cache file (CPU), and tuning itself (GPU)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

KEY_SCRIPT = (
    "import sys; sys.path.insert(0, sys.argv[1]);"
    "from paper_1412_7228_amd import autotune as t;"
    "print(t.batch_key('dev', [(64, 64), (100, 37), (512, 300)], dict(precision='fp32', eos='cs')))"
)


def test_batch_key_is_the_same_in_every_process():
    keys = set()
    for seed in ("1", "2", "12345"):
        env = dict(os.environ, PYTHONHASHSEED=seed)
        out = subprocess.run([sys.executable, "-c", KEY_SCRIPT, ROOT], capture_output=True, text=True,
                             env=env, check=True).stdout.strip()
        keys.add(out)
    assert len(keys) == 1
    from paper_1412_7228_amd import autotune as t

    k = keys.pop()
    # the order of the domains does not matter, their sizes do
    assert k == t.batch_key("dev", [(512, 300), (64, 64), (100, 37)], dict(precision="fp32", eos="cs"))
    assert k != t.batch_key("dev", [(64, 64), (100, 38), (512, 300)], dict(precision="fp32", eos="cs"))


def test_cache_round_trip(tmp_path, monkeypatch):
    from paper_1412_7228_amd import autotune as t

    monkeypatch.setenv("LBM_TUNE_CACHE", str(tmp_path / "sub" / "tune.json"))
    assert t._load() == {}
    t._store({"k": {"tile": [128, 8, 2], "ms": 0.1}})
    assert t._load() == {"k": {"tile": [128, 8, 2], "ms": 0.1}}
    (tmp_path / "sub" / "tune.json").write_text("not json")
    assert t._load() == {}


@pytest.mark.gpu
def test_tuning_picks_a_candidate_caches_it_and_keeps_the_state(tmp_path, monkeypatch):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device visible")
    from paper_1412_7228_amd import autotune as t, inputs, lbm

    print("[gpu-case] autotune lattice + batch", flush=True)
    monkeypatch.setenv("LBM_TUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = dict(nx=300, ny=120, eos="cs", T_over_Tc=0.7, A=-0.5, kappa=0.2, precision="fp32")
    rho = inputs.spinodal(300, 120, 0.183713, noise=1e-2, seed=1)
    cands = [(256, 16, 2), (128, 8, 2), (64, 32, 1)]
    a, b = lbm.Lattice(cfg), lbm.Lattice(cfg)
    a.init_field(rho)
    b.init_field(rho)
    res = t.tune_lattice(a, steps=8, candidates=cands)
    assert tuple(res["tile"]) in cands and len(res["table"]) == 3
    # the tuning advanced the state by its timing steps; the bits do not depend on the shape
    b.step(a.info()["step"])
    assert np.array_equal(a.f_soa(), b.f_soa())
    again = t.tune_lattice(a, candidates=cands)  # from the cache: no timing
    assert again["tile"] == res["tile"] and tuple(a.launch) == tuple(res["tile"])
    assert json.loads((tmp_path / "tune.json").read_text())
    bcfgs = [dict(cfg, nx=n, ny=n) for n in (64, 100, 150)]
    batch = lbm.Batch(bcfgs)
    for i, c in enumerate(bcfgs):
        batch.init_field(i, inputs.spinodal(c["nx"], c["ny"], 0.183713, noise=1e-2, seed=i))
    bres = t.tune_batch(batch, steps=4, candidates=[("per_step", 128, 16, 2), ("per_step", 64, 16, 1)])
    assert len(bres["table"]) == 2 and batch.launch["steps_per_pass"] == bres["launch"][3]
    assert all(o["n_nonfinite"] == 0 for o in batch.observables())
