"""Row-range launches (lbm_step_rows) and the y-slab decomposition they allow, on one GPU.

The periodic lattice is the paper's domain (Sec. 3.1.1).  Cut into S slabs of h
rows, each slab a context of h + 4n rows whose first and last 2n rows are ghost
rows, advanced one launch at a time with lbm_step_rows(n, 2n, h) and the ghost
rows copied from the neighbouring slabs' current buffers after each launch, the
slabs hold exactly (bit for bit) the rows of the undivided lattice: the per-cell
arithmetic does not depend on the tile a cell falls in.
"""
import numpy as np
import pytest

from paper_1412_7228_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device visible")
    from paper_1412_7228_amd import lbm as mod

    mod.load_library()  # with a HIP device visible the library must load: no fallback
    return mod


def say(msg):
    print(f"[slabs] {msg}", flush=True)


def _cfg(nx, ny, precision):
    return dict(nx=nx, ny=ny, eos="cs", T_over_Tc=0.7, A=-0.5, kappa=0.3, precision=precision)


def _lattice(lbm, cfg, n):
    lat = lbm.Lattice(cfg)
    lat.set_launch(0, 0, n)
    return lat


@pytest.mark.parametrize("precision,n,nx,S,h,split", [
    ("fp32", 2, 300, 4, 24, False),  # several strips, ragged last strip
    ("fp64", 2, 130, 3, 20, False),
    ("fp32", 1, 200, 4, 13, False),  # one step per launch, ragged row blocks
    ("fp32", 2, 260, 2, 7, False),   # slabs thinner than a tile
    ("fp32", 2, 140, 1, 30, False),  # one slab: its own neighbour on both sides
    ("fp32", 2, 300, 4, 24, True),   # interior rows first, then the rows next to the ghosts
    ("fp64", 2, 130, 3, 20, True),
    ("fp32", 1, 200, 4, 13, True),
])
def test_slabs_with_ghost_rows_equal_periodic_lattice(lbm, precision, n, nx, S, h, split):
    import torch

    say(f"{precision} n={n} nx={nx} slabs={S} x {h} rows split={split}")
    NY, g = S * h, 2 * n
    rho = inputs.spinodal(nx, NY, 0.183713, noise=1e-2, seed=5)
    lat = _lattice(lbm, _cfg(nx, NY, precision), n)
    lat.init_field(rho)
    lat.step(2 * n)  # a state that is not the initial equilibrium
    slabs = []
    full = lat.state_tensor()
    for s in range(S):
        sl = _lattice(lbm, _cfg(nx, h + 2 * g, precision), n)
        sl.init_field(np.full((h + 2 * g, nx), 0.2))
        rows = torch.tensor([(s * h - g + r) % NY for r in range(h + 2 * g)], device=full.device)
        sl.state_tensor().copy_(full.index_select(1, rows))
        slabs.append(sl)

    def refresh():
        # ghost rows of every slab's current buffer from its neighbours' interior rows
        cur = [sl.state_tensor() for sl in slabs]
        new = [c.clone() for c in cur]
        for s in range(S):
            new[s][:, :g] = cur[(s - 1) % S][:, h:h + g]
            new[s][:, h + g:] = cur[(s + 1) % S][:, g:2 * g]
        for c, m in zip(cur, new):
            c.copy_(m)

    for launch in range(5):
        lat.step(n)
        if split:
            # the ghost rows have not arrived yet: the rows that read none of them go first
            for sl in slabs:
                t = sl.state_tensor()
                t[:, :g] = float("nan")
                t[:, h + g:] = float("nan")
                sl.step_rows(n, 2 * g, h - 2 * g, more=True)
            refresh()
            for sl in slabs:
                sl.step_rows(n, g, g, more=True)
                sl.step_rows(n, h, g)
        else:
            for sl in slabs:
                sl.step_rows(n, g, h)
            refresh()
        full = lat.state_tensor()
        for s in range(S):
            a = slabs[s].state_tensor()[:, g:g + h, :nx]
            b = full[:, s * h:(s + 1) * h, :nx]
            assert torch.equal(a, b), f"slab {s} differs after launch {launch}"
    for sl in slabs:
        sl.close()
    lat.close()


@pytest.mark.parametrize("n", [1, 2])
def test_full_row_range_equals_step(lbm, n):
    import torch

    say(f"full range n={n}")
    nx, ny = 270, 50
    rho = inputs.spinodal(nx, ny, 0.183713, noise=1e-2, seed=6)
    a = _lattice(lbm, _cfg(nx, ny, "fp32"), n)
    b = _lattice(lbm, _cfg(nx, ny, "fp32"), n)
    a.init_field(rho)
    b.init_field(rho)
    for _ in range(3):
        a.step(n)
        b.step_rows(n, 0, ny)
    assert a.info()["step"] == b.info()["step"] == 3 * n
    assert torch.equal(a.state_tensor()[:, :, :nx], b.state_tensor()[:, :, :nx])


def test_partial_range_leaves_other_rows(lbm):
    """A launch over rows [10, 22) writes those rows of the step it computes and
    leaves the other rows of the destination buffer as they were (here: the
    initial state, written two launches earlier)."""
    import torch

    say("partial range keeps other rows")
    nx, ny = 200, 40
    rho = inputs.spinodal(nx, ny, 0.183713, noise=1e-2, seed=7)
    lat = _lattice(lbm, _cfg(nx, ny, "fp32"), 2)
    ref = _lattice(lbm, _cfg(nx, ny, "fp32"), 2)
    lat.init_field(rho)
    ref.init_field(rho)
    start = lat.state_tensor().clone()
    lat.step_rows(2, 0, ny)
    lat.step_rows(2, 10, 12)
    ref.step(4)
    now, want = lat.state_tensor(), ref.state_tensor()
    assert torch.equal(now[:, :10], start[:, :10]) and torch.equal(now[:, 22:], start[:, 22:])
    assert torch.equal(now[:, 10:22, :nx], want[:, 10:22, :nx])


def test_step_rows_rejects_bad_arguments(lbm):
    say("argument checks")
    lat = _lattice(lbm, _cfg(130, 30, "fp32"), 2)
    with pytest.raises(lbm.LBMError):
        lat.step_rows(1, 0, 10)  # before init
    lat.init_field(np.full((30, 130), 0.2))
    for n, y0, rows in ((3, 0, 10), (0, 0, 10), (2, -1, 10), (2, 25, 6), (2, 5, 0)):
        with pytest.raises(lbm.LBMError):
            lat.step_rows(n, y0, rows)
    one = _lattice(lbm, _cfg(130, 30, "fp32"), 1)
    one.init_field(np.full((30, 130), 0.2))
    with pytest.raises(lbm.LBMError):
        one.step_rows(2, 0, 30)  # two steps need two steps per pass
    one.step_rows(1, 0, 30)


def test_open_row_range_launch_state_rules(lbm):
    """While a row-range launch is open (more ranges of the same steps to come), the
    source buffer stays current, lbm_step and set_launch are refused, another step
    count is refused, and the closing call makes the destination current."""
    say("open row-range launch")
    lat = _lattice(lbm, _cfg(130, 30, "fp32"), 2)
    lat.init_field(np.full((30, 130), 0.2))
    before = lat.info()
    lat.step_rows(2, 0, 10, more=True)
    assert lat.info() == before  # still the source buffer and the same step
    with pytest.raises(lbm.LBMError):
        lat.step(2)
    with pytest.raises(lbm.LBMError):
        lat.set_launch(0, 0, 1)
    with pytest.raises(lbm.LBMError):
        lat.step_rows(1, 10, 10)
    lat.step_rows(2, 10, 20)
    after = lat.info()
    assert after["step"] == 2 and after["f_cur"] != before["f_cur"]
    lat.step(2)  # allowed again


@pytest.mark.parametrize("precision,nx,S,h", [("fp32", 300, 4, 24), ("fp64", 130, 2, 20)])
def test_deep_ghost_zone_two_launches_per_exchange(lbm, precision, nx, S, h):
    """Slabs with 8 ghost rows per side exchange once per two launches of two steps:
    the first launch also updates the inner 4 ghost rows on each side (rows [4, h + 12)),
    the second only the slab (rows [8, h + 8)); the slabs then hold the periodic
    lattice's rows bit for bit."""
    import torch

    say(f"deep ghost zone {precision} {S} slabs x {h} rows")
    NY, g = S * h, 8
    rho = inputs.spinodal(nx, NY, 0.183713, noise=1e-2, seed=11)
    lat = _lattice(lbm, _cfg(nx, NY, precision), 2)
    lat.init_field(rho)
    full = lat.state_tensor()
    slabs = []
    for s in range(S):
        sl = _lattice(lbm, _cfg(nx, h + 2 * g, precision), 2)
        sl.init_field(np.full((h + 2 * g, nx), 0.2))
        rows = torch.tensor([(s * h - g + r) % NY for r in range(h + 2 * g)], device=full.device)
        sl.state_tensor().copy_(full.index_select(1, rows))
        slabs.append(sl)
    for exchange in range(3):
        lat.step(4)
        for sl in slabs:
            sl.step_rows(2, 4, h + 8)
            sl.step_rows(2, 8, h)
        cur = [sl.state_tensor() for sl in slabs]
        new = [c.clone() for c in cur]
        for s in range(S):
            new[s][:, :g] = cur[(s - 1) % S][:, h:h + g]
            new[s][:, h + g:] = cur[(s + 1) % S][:, g:2 * g]
        for c, m in zip(cur, new):
            c.copy_(m)
        full = lat.state_tensor()
        for s in range(S):
            assert torch.equal(slabs[s].state_tensor()[:, g:g + h, :nx], full[:, s * h:(s + 1) * h, :nx]), \
                (s, exchange)
