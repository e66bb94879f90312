"""lbm_observables_noalloc (the observables entry point that allocates nothing) against
lbm_observables, through the C ABI: two calls in a row, the second on a smaller lattice of
another EOS and precision, then the first again; a state with U > 0 cells; and the size
limit.  The two entry points run the same per-cell arithmetic and the same fixed-order
reduction, so every observable must agree bit for bit."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import thermo as th
from paper_1412_7228_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("step", "mass", "mom_x", "mom_y", "rho_min", "rho_max", "rho_in", "rho_out", "p_in", "p_out",
        "dp", "R_e", "sigma", "max_u", "n_nonfinite", "n_domain", "status")


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


def droplet_lattice(lbm, cfg, R, steps, seed):
    e = th.carnahan_starling() if cfg["eos"] == "cs" else th.vdw(cfg.get("K", 0.3))
    _, Tc = th.critical_point(e)
    rv, rl = th.maxwell(e, cfg["T_over_Tc"] * Tc)
    lat = lbm.Lattice(cfg)
    lat.init_field(inputs.droplet(cfg["nx"], cfg["ny"], R, rl, rv, W=4.0, noise=1e-2, seed=seed))
    lat.step(steps)
    return lat


def assert_same(a, b, label):
    for k in KEYS:
        va, vb = a[k], b[k]
        same = (va == vb) or (isinstance(va, float) and np.isnan(va) and np.isnan(vb))
        assert same, (label, k, va, vb)


def test_noalloc_observables_equal_the_allocating_call(lbm):
    big = dict(nx=300, ny=201, eos="cs", T_over_Tc=0.75, A=-0.6, kappa=0.4, precision="fp32")
    small = dict(nx=37, ny=23, eos="vdw", K=0.3, T_over_Tc=0.9, A=0.3, kappa=0.7, precision="fp64")
    say("noalloc observables: 300x201 fp32 cs, 50 steps")
    lat1 = droplet_lattice(lbm, big, 60, 50, seed=4)
    first = lat1.observables(noalloc=True)
    assert_same(first, lat1.observables(), "300x201 fp32")
    assert first["step"] == 50 and first["mass"] > 0 and first["status"] == 0
    say("noalloc observables: 37x23 fp64 vdw, 31 steps (smaller, after the larger one)")
    lat2 = droplet_lattice(lbm, small, 8, 31, seed=5)
    second = lat2.observables(noalloc=True)
    ref2 = lat2.observables()
    assert_same(second, ref2, "37x23 fp64")
    # nothing of the larger lattice's partial sums leaks into the smaller one
    assert abs(second["mass"] / lat2.field("rho").sum() - 1) < 1e-13
    say("noalloc observables: the larger lattice again, 7 more steps")
    lat1.step(7)
    assert_same(lat1.observables(noalloc=True), lat1.observables(), "300x201 fp32 again")
    lat1.close()
    lat2.close()


def test_noalloc_observables_report_faults_like_the_allocating_call(lbm):
    say("noalloc observables: U > 0 cells, 48x40 fp64, 3 steps")
    cfg = dict(nx=48, ny=40, eos="cs", T_over_Tc=0.8, A=-0.5, kappa=0.3, precision="fp64")
    lat = lbm.Lattice(cfg)
    lat.init_field(inputs.droplet(48, 40, 8, 0.5, 0.03, W=4.0, noise=0.0))
    lat.step(3)
    na = lat.observables(check=False, noalloc=True)
    ref = lat.observables(check=False)
    assert na["status"] == ref["status"] == -5 and na["n_domain"] > 0
    assert_same(na, ref, "U>0 48x40")
    lat.close()


def test_noalloc_observables_size_limit(lbm):
    lib = lbm.load_library()
    limit = lib.lbm_noalloc_max_cells()
    assert limit == 2**28
    say("noalloc observables: a lattice one row above the limit is refused before anything else")
    lat = lbm.Lattice(dict(nx=16384, ny=16385, eos="cs", precision="fp32"), torch_buffers=False)
    o = lbm.Obs()
    st = lib.lbm_observables_noalloc(lat.h, ctypes.byref(o))
    assert st == -1 and b"exceed" in lib.lbm_last_error()
    lat.close()
