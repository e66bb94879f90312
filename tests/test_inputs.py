"""The seeded input generators: same seed, same arrays; the recipes' shapes, ranges and
profiles as documented (a droplet centred at (nx/2, ny/2) with the tanh profile, the
uneven batch draws inside their ranges)."""
import numpy as np

from paper_1412_7228_amd import inputs


def test_same_seed_same_arrays_other_seed_other_arrays():
    a = inputs.spinodal(50, 40, 0.2, noise=1e-2, seed=7)
    b = inputs.spinodal(50, 40, 0.2, noise=1e-2, seed=7)
    c = inputs.spinodal(50, 40, 0.2, noise=1e-2, seed=8)
    assert a.shape == (40, 50) and np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.all(np.abs(a / 0.2 - 1) <= 1e-2)
    assert abs(a.mean() / 0.2 - 1) < 2e-3


def test_droplet_profile():
    rl, rv, R, W = 0.3, 0.02, 12.0, 5.0
    rho = inputs.droplet(64, 48, R, rl, rv, W=W, noise=0.0)
    assert rho.shape == (48, 64)
    # centre and far corner, and the midpoint density at distance R from the centre
    prof = lambda r: 0.5 * (rl + rv) - 0.5 * (rl - rv) * np.tanh(2.0 * (r - R) / W)
    assert abs(rho[24, 32] - prof(0.0)) < 1e-15 and abs(rho[0, 0] - prof(np.hypot(32, 24))) < 1e-15
    assert abs(rho[24, 32] - rl) < 1e-3 * (rl - rv) and abs(rho[0, 0] - rv) < 1e-6
    mid = 0.5 * (rl + rv)
    assert abs(rho[24, 32 + 12] - mid) < 1e-12
    # monotone along a ray out of the centre
    assert np.all(np.diff(rho[24, 32:]) <= 0)


def test_slab_and_taylor_green():
    s = inputs.slab(100, 4, 0.3, 0.02, W=5.0, noise=0.0)
    assert s.shape == (4, 100) and np.allclose(s[0], s[3])
    assert abs(s[0, 50] - 0.3) < 1e-6 and abs(s[0, 0] - 0.02) < 1e-6
    rho, ux, uy = inputs.taylor_green(16, u0=1e-3)
    assert np.all(rho == 1.0)
    # divergence-free on the lattice to round-off (central differences of the closed form)
    div = (np.roll(ux, -1, 1) - np.roll(ux, 1, 1)) + (np.roll(uy, -1, 0) - np.roll(uy, 1, 0))
    assert np.abs(div).max() < 1e-15


def test_batch_draws_in_range_and_seeded():
    d = inputs.batch_draws(256, 3)
    assert d == inputs.batch_draws(256, 3) and d != inputs.batch_draws(256, 4)
    for x in d:
        assert 64 <= x["nx"] == x["ny"] <= 512
        assert 0.15 * x["nx"] <= x["R"] <= 0.35 * x["nx"]
        assert 0.6 <= x["T_over_Tc"] <= 0.85 and 0.0 <= x["kappa"] <= 0.8 and -0.7 <= x["A"] <= -0.3
    sides = np.array([x["nx"] for x in d])
    assert sides.min() < 100 and sides.max() > 450  # spans the range


def test_batch_draws_are_the_head_of_the_seeded_stream():
    """The redraw of infeasible draws continues the same seeded stream: batch_draws(n) is
    its first n draws, and draws are numbered along it."""
    import itertools

    d = inputs.batch_draws(40, 3)
    s = list(itertools.islice(inputs.batch_draw_stream(3), 60))
    assert d == s[:40]
    assert [x["index"] for x in s] == list(range(60))
    assert s[40:] != list(itertools.islice(inputs.batch_draw_stream(4), 40, 60))
