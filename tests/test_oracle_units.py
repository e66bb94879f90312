"""Pins of the oracle's building blocks: transform, collision, force and tensor Q.

Each pin is a closed form, a textbook reduction or a Taylor expansion that a
plausible mistake in the oracle (wrong row of M, dropped source term, wrong
weight, sign or prefactor) would break.
"""
import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def hermite_feq(rho, ux, uy):
    eu = EX * ux + EY * uy
    return W * rho * (1 + 3 * eu + 4.5 * eu**2 - 1.5 * (ux * ux + uy * uy))


def guo_source(ux, uy, Fx, Fy):
    """Guo, Zheng & Shi (2002) forcing term without the (1 - 1/2tau) prefactor."""
    eu = EX * ux + EY * uy
    return W * (3 * ((EX - ux) * Fx + (EY - uy) * Fy) + 9 * eu * (EX * Fx + EY * Fy))


def test_moment_matrix_orthogonality(oracle_mod):
    M, Minv = oracle_mod.moment_matrix()
    # Lallemand & Luo (2000): the D2Q9 rows are orthogonal with squared norms
    assert np.array_equal(M @ M.T, np.diag([9.0, 36, 36, 6, 12, 6, 12, 4, 4]))
    assert np.abs(Minv @ M - np.eye(9)).max() < 1e-15
    # integer entries
    assert np.array_equal(M, np.round(M))


def test_moments_of_equilibrium_are_eq4(oracle_mod):
    M, _ = oracle_mod.moment_matrix()
    g = np.random.default_rng(1)
    for _ in range(20):
        rho, ux, uy = g.uniform(0.1, 3), g.uniform(-0.2, 0.2), g.uniform(-0.2, 0.2)
        m = M @ hermite_feq(rho, ux, uy)
        v2 = ux * ux + uy * uy
        eq4 = rho * np.array([1, -2 + 3 * v2, 1 - 3 * v2, ux, -ux, uy, -uy, ux * ux - uy * uy, ux * uy])
        assert np.abs(m - eq4).max() < 1e-14 * max(1, rho)


def _cfg(**kw):
    c = dict(nx=3, ny=3, eos="ideal")
    c.update(kw)
    return c


@pytest.mark.parametrize("s", [0.6, 1.0, 1.3, 1.85])
def test_equal_rates_reduce_to_bgk_with_guo_forcing(oracle_mod, s):
    """All rates equal: MRT with the (I - Lambda/2) S source is BGK with Guo forcing."""
    o = oracle_mod.Oracle(_cfg(s_e=s, s_eps=s, s_q=s, s_nu=s))
    g = np.random.default_rng(7)
    for _ in range(10):
        f = hermite_feq(g.uniform(0.5, 2), g.uniform(-0.1, 0.1), g.uniform(-0.1, 0.1))
        f = f * (1 + 0.05 * g.uniform(-1, 1, 9))
        Fx, Fy = g.uniform(-0.01, 0.01, 2)
        rho = f.sum()
        ux = (f @ EX + Fx / 2) / rho
        uy = (f @ EY + Fy / 2) / rho
        bgk = f - s * (f - hermite_feq(rho, ux, uy)) + (1 - s / 2) * guo_source(ux, uy, Fx, Fy)
        got = o.collide_cell(f, (Fx, Fy))
        assert np.abs(got - bgk).max() < 2e-16 * 20


def test_collision_conserves_mass_and_adds_force(oracle_mod):
    o = oracle_mod.Oracle(_cfg(s_e=1.3, s_eps=0.7, s_q=1.1, s_nu=1.6))
    g = np.random.default_rng(3)
    f = hermite_feq(1.2, 0.03, -0.02) * (1 + 0.1 * g.uniform(-1, 1, 9))
    F = (1e-3, -2e-3)
    out = o.collide_cell(f, F, (1e-3, -5e-4, 2e-4))
    assert abs(out.sum() - f.sum()) < 1e-15
    assert abs(out @ EX - (f @ EX + F[0])) < 1e-15
    assert abs(out @ EY - (f @ EY + F[1])) < 1e-15


def test_Q_term_shifts_momentum_flux(oracle_mod):
    """With s_e = s_nu = 1, the C source of Eq. (26) changes the post-collision momentum
    flux by (3/4) tr(Q) I - Q: its deviatoric part is -Q, which cancels the (1-kappa)
    surface-tension part while leaving the normal pressure alone (Eq. 28)."""
    o = oracle_mod.Oracle(_cfg(s_e=1.0, s_nu=1.0, s_eps=0.8, s_q=1.2))
    f = hermite_feq(1.0, 0.01, 0.02)
    Q = np.array([2e-3, -7e-4, 5e-4])
    d = o.collide_cell(f, (0, 0), Q) - o.collide_cell(f, (0, 0))
    Pxx, Pyy, Pxy = d @ (EX * EX), d @ (EY * EY), d @ (EX * EY)
    tr = Q[0] + Q[1]
    assert abs(Pxx - (0.75 * tr - Q[0])) < 2e-15
    assert abs(Pyy - (0.75 * tr - Q[1])) < 2e-15
    assert abs(Pxy - (-Q[2])) < 2e-15
    assert abs(d.sum()) < 2e-15 and abs(d @ EX) < 2e-15 and abs(d @ EY) < 2e-15


# ---------------------------------------------------------------------------
# Force (Eq. 9) and Q (Eq. 23) against their Taylor expansions on smooth fields
# ---------------------------------------------------------------------------
def _smooth_fields(oracle_mod, n, A, kappa=1.0, G=-1.0):
    """A smooth periodic density on an n x n lattice, CS EOS at 0.8Tc, and the
    analytic psi and its derivatives up to third order (through the EOS)."""
    cfg = dict(nx=n, ny=n, eos="cs", T_over_Tc=0.8, A=A, kappa=kappa, G=G)
    o = oracle_mod.Oracle(cfg)
    e = oracle_mod.eos_of(cfg)
    T = o.T
    k = 2 * np.pi / n
    y, x = np.mgrid[0:n, 0:n].astype(float)
    # psi itself is the smooth test field; rho follows from inverting psi(rho)
    from scipy import optimize

    psi = 0.12 + 0.03 * np.sin(k * x + 0.3) * np.cos(2 * k * y + 0.1) + 0.02 * np.cos(k * y)
    rho_of = {}
    flat = psi.ravel()
    rho = np.empty_like(flat)
    for i, s in enumerate(flat):
        if s not in rho_of:
            rho_of[s] = optimize.brentq(lambda r: np.sqrt(max(0.0, 2 * (float(e.p(r, T)) - r / 3) / G)) - s,
                                        1e-6, 0.0943, xtol=1e-16, rtol=1e-15)
        rho[i] = rho_of[s]
    rho = rho.reshape(psi.shape)
    # analytic derivatives of psi
    px = 0.03 * k * np.cos(k * x + 0.3) * np.cos(2 * k * y + 0.1)
    py = -0.06 * k * np.sin(k * x + 0.3) * np.sin(2 * k * y + 0.1) - 0.02 * k * np.sin(k * y)
    pxx = -0.03 * k * k * np.sin(k * x + 0.3) * np.cos(2 * k * y + 0.1)
    pyy = -0.12 * k * k * np.sin(k * x + 0.3) * np.cos(2 * k * y + 0.1) - 0.02 * k * k * np.cos(k * y)
    pxy = -0.06 * k * k * np.cos(k * x + 0.3) * np.sin(2 * k * y + 0.1)
    lap = pxx + pyy
    # gradient of the Laplacian
    lx = -0.03 * k**3 * np.cos(k * x + 0.3) * np.cos(2 * k * y + 0.1) * 5
    ly = (0.03 * 4 * k**3 * np.sin(k * x + 0.3) * np.sin(2 * k * y + 0.1) * 5 / 2
          + 0.02 * k**3 * np.sin(k * y))
    # d/dy of [-(0.03*5) k^2 sin cos(2ky)] = 0.03*5*2 k^3 sin(kx) sin(2ky); d/dy of -0.02k^2 cos(ky) = 0.02 k^3 sin(ky)
    d = dict(psi=psi, px=px, py=py, pxx=pxx, pyy=pyy, pxy=pxy, lap=lap, lx=lx, ly=ly)
    return o, rho, d


@pytest.mark.parametrize("A", [-0.5, 0.0, 0.6, 1.0])
def test_force_leading_order_eq11(oracle_mod, A):
    """F = -G psi grad psi + O(k^3): halving k cuts the remainder by 8 relative to k^1 terms.

    The next order is also checked: from the isotropy of the weights,
    sum_a w_a phi(x+e_a) e_a = grad phi + (1/6) grad lap phi + O(k^5), so
    F = -G [psi grad psi + (1/6) psi grad lap psi + (A/6)(lap psi grad psi + grad |grad psi|^2)] + O(k^5).
    """
    G = -1.0
    errs1, errs2 = [], []
    for n in (32, 64):
        o, rho, d = _smooth_fields(oracle_mod, n, A, G=G)
        got = o.interaction(rho)
        assert np.abs(got["psi"] - d["psi"]).max() < 1e-12
        lead_x = -G * d["psi"] * d["px"]
        lead_y = -G * d["psi"] * d["py"]
        # grad |grad psi|^2 = 2 (px pxx + py pxy, px pxy + py pyy)
        gx = 2 * (d["px"] * d["pxx"] + d["py"] * d["pxy"])
        gy = 2 * (d["px"] * d["pxy"] + d["py"] * d["pyy"])
        nxt_x = -G * (d["psi"] * d["lx"] / 6 + A / 6 * (d["lap"] * d["px"] + gx))
        nxt_y = -G * (d["psi"] * d["ly"] / 6 + A / 6 * (d["lap"] * d["py"] + gy))
        scale = np.abs(lead_x).max()
        errs1.append(max(np.abs(got["Fx"] - lead_x).max(), np.abs(got["Fy"] - lead_y).max()) / scale)
        errs2.append(max(np.abs(got["Fx"] - lead_x - nxt_x).max(),
                         np.abs(got["Fy"] - lead_y - nxt_y).max()) / scale)
    # leading remainder is O(k^2) relative, the next one O(k^4)
    assert 3.5 < errs1[0] / errs1[1] < 4.5
    assert 14 < errs2[0] / errs2[1] < 18
    assert errs2[1] < 2e-4


@pytest.mark.parametrize("A", [-0.5, 0.0, 0.7])
def test_Q_leading_order_eq24(oracle_mod, A):
    """Q -> kappa[(G/12)(psi lap psi + A |grad psi|^2) I + (G/6)(psi grad grad psi + A grad psi grad psi)]."""
    G, kappa = -1.0, 0.8
    errs = []
    for n in (32, 64):
        o, rho, d = _smooth_fields(oracle_mod, n, A, kappa=kappa, G=G)
        got = o.interaction(rho)
        g2 = d["px"] ** 2 + d["py"] ** 2
        iso = G / 12 * (d["psi"] * d["lap"] + A * g2)
        qxx = kappa * (iso + G / 6 * (d["psi"] * d["pxx"] + A * d["px"] ** 2))
        qyy = kappa * (iso + G / 6 * (d["psi"] * d["pyy"] + A * d["py"] ** 2))
        qxy = kappa * (G / 6 * (d["psi"] * d["pxy"] + A * d["px"] * d["py"]))
        scale = np.abs(qxx).max()
        errs.append(max(np.abs(got["Qxx"] - qxx).max(), np.abs(got["Qyy"] - qyy).max(),
                        np.abs(got["Qxy"] - qxy).max()) / scale)
    assert 3.5 < errs[0] / errs[1] < 4.5
    assert errs[1] < 2e-2


def test_force_sums_to_zero_on_periodic_lattice(oracle_mod):
    """Eq. (9) is a pair interaction on a periodic lattice: sum_x F = 0 (momentum)."""
    g = np.random.default_rng(11)
    for A in (-0.9, -0.3, 0.4, 1.0):
        o = oracle_mod.Oracle(dict(nx=17, ny=11, eos="cs", T_over_Tc=0.7, A=A))
        rho = g.uniform(0.01, 0.35, (11, 17))
        got = o.interaction(rho)
        scale = np.abs(got["Fx"]).max()
        assert abs(got["Fx"].sum()) < 1e-14 * scale * rho.size
        assert abs(got["Fy"].sum()) < 1e-14 * scale * rho.size


def test_ideal_gas_has_no_interaction(oracle_mod):
    o = oracle_mod.Oracle(dict(nx=5, ny=4, eos="ideal", A=-0.5, kappa=0.7))
    got = o.interaction(np.random.default_rng(0).uniform(0.5, 1.5, (4, 5)))
    for k in ("U", "psi", "Fx", "Fy", "Qxx", "Qyy", "Qxy"):
        assert np.abs(got[k]).max() < 1e-16


def test_laplace_fit_exact_line_least_squares_and_spread(oracle_mod):
    """Eq. (22) over drop sizes: drops that obey dp = sigma / R exactly give sigma back
    with zero spread; scattered drops give the slope that numpy's least squares finds
    for the model dp = sigma x, x = 1/R; drops whose dp R are (0.9, 1, 1.1) sigma have a
    spread of 0.2; a single drop gives dp R."""
    R = np.array([20.0, 30.0, 40.0, 50.0, 60.0])
    s, spread = oracle_mod.laplace_fit(0.0123 / R, R)
    assert abs(s / 0.0123 - 1) < 1e-14 and spread < 1e-14
    dp = 0.0123 / R * (1 + 0.05 * np.random.default_rng(5).standard_normal(R.size))
    want = np.linalg.lstsq((1.0 / R)[:, None], dp, rcond=None)[0][0]
    assert abs(oracle_mod.laplace_fit(dp, R)[0] / want - 1) < 1e-13
    _, spread = oracle_mod.laplace_fit(np.array([0.9, 1.0, 1.1]) * 0.01 / R[:3], R[:3])
    assert abs(spread - 0.2) < 1e-13
    s, spread = oracle_mod.laplace_fit([2e-4], [25.0])
    assert abs(s / (2e-4 * 25.0) - 1) < 1e-15 and spread == 0.0
    for bad in (([], []), ([1e-3], [0.0]), ([1e-3, 2e-3], [20.0])):
        with pytest.raises(ValueError):
            oracle_mod.laplace_fit(*bad)


@pytest.mark.parametrize("eos,tr,rhos", [
    ("cs", 0.8, np.linspace(0.005, 0.6, 24)),
    ("vdw", 0.9, np.linspace(0.2, 9.0, 24)),
    ("pr", 0.8, np.linspace(0.01, 8.5, 24)),
    ("pr", 0.6, np.linspace(0.01, 9.0, 24)),
    ("ideal", 0.0, np.linspace(0.1, 3.0, 24)),
])
def test_c_pressure_equals_thermo_pressure(oracle_mod, eos, tr, rhos):
    """The C oracle's K p_EOS (used in every density pass) is the same function as the
    thermodynamics module's (whose critical point, Maxwell construction and, for PR, the
    acentric factor are pinned in the thermodynamics tests): every EOS at 24 densities
    across both phases, with K = 0.5, to 1e-14 of the size of the pressure's two terms,
    K (rho R T + a rho^2) (the pressure passes through zero between the phases, where the
    terms cancel and a relative difference says nothing)."""
    from oracle import thermo as th

    cfg = dict(nx=3, ny=3, eos=eos, K=0.5, T_over_Tc=tr if tr else 0.8)
    o = oracle_mod.Oracle(cfg)
    if eos == "ideal":
        want = rhos / 3.0
        scale = want
    else:
        e = oracle_mod.eos_of(cfg)
        T, Tc = oracle_mod.temperature(cfg)
        want = np.asarray(e.p(rhos, T, Tc))
        assert isinstance(e, th.EOS) and e.K == 0.5
        scale = e.K * (rhos * e.R * T + e.a * rhos**2)
    got = np.array([o.pressure(r) for r in rhos])
    assert (np.abs(got - want) <= 1e-14 * scale).all(), np.max(np.abs(got - want) / scale)


def test_initial_equilibrium_has_the_moments_of_eq4(oracle_mod):
    """The oracle's initial state (orc_init_equilibrium, the second-order equilibrium in
    velocity space) transformed by M equals the equilibrium moments of Eq. (4) written in
    moment space, rho (1, -2 + 3|u|^2, 1 - 3|u|^2, ux, -ux, uy, -uy, ux^2 - uy^2, ux uy),
    to 1e-14, including the velocity terms, at |u| up to about 0.14."""
    M, _ = oracle_mod.moment_matrix()
    g = np.random.default_rng(11)
    n = 6
    o = oracle_mod.Oracle(dict(nx=n, ny=n, eos="ideal"))
    rho = g.uniform(0.05, 3.0, (n, n))
    ux = g.uniform(-0.1, 0.1, (n, n))
    uy = g.uniform(-0.1, 0.1, (n, n))
    o.init_field(rho, ux, uy)
    m = np.einsum("ka,yxa->yxk", M, o.f)
    v2 = ux * ux + uy * uy
    eq4 = rho[..., None] * np.stack([np.ones_like(ux), -2 + 3 * v2, 1 - 3 * v2, ux, -ux, uy, -uy,
                                     ux * ux - uy * uy, ux * uy], axis=-1)
    assert np.abs(m - eq4).max() < 1e-14 * rho.max()
    # and the moments do not vanish: the test sees the velocity terms
    assert np.abs(eq4[..., 3]).max() > 0.1 and np.abs(eq4[..., 8]).max() > 1e-3
    # the read-out inverts it: v = (sum f e + F/2)/rho with F = 0 for the ideal gas
    fl = o.fields()
    assert np.abs(fl["ux"] - ux).max() < 1e-15 and np.abs(fl["uy"] - uy).max() < 1e-15
