"""Host-side thermodynamics of the pseudo-potential model (FP64, numpy/scipy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the tests, the entry point's smoke check and the CPU-baseline leg of the
benchmark may use anything under ``oracle/``.

What is here, each a plain definition written out:

* equations of state: van der Waals (Sec. 3, Eq. 21), Peng-Robinson (Sec. 4,
  Eq. 29) and Carnahan-Starling (not in the paper; the usual a=1, b=4, R=1
  form), each multiplied by the stability factor K of Eq. (21);
* the critical point (dp/drho = d2p/drho2 = 0) and the Maxwell equal-area
  construction (textbook thermodynamics);
* the mechanical stability condition, Eq. (17), with eps = -2a/b and
  a = 3A, b = 3 (Sec. 2, text under Eq. 16), i.e. eps = -2A;
* the leading-order surface tension of Eq. (20), multiplied by (1 - kappa)
  as Eq. (28) states, with (dpsi/dn)^2 obtained from P_xx = p_c (Eq. 14);
* the exact steady balance of the discrete model for a flat interface
  (derived here from Eqs. 1, 9, 23, 25 and 26, not printed in the paper):
  with s_e = s_nu = 1 a 1-D steady state obeys
      rho(x+1) - rho(x) = 3/2 [F(x) + F(x+1)],
      F(x) = -(A/2)[U(x+1) - U(x-1)] - (1-A)(G/2) psi(x)[psi(x+1) - psi(x-1)],
  independent of kappa.  This is what makes Table 1's densities exact.

The pseudo-potential convention (Eq. 10 with c = 1, c_s^2 = 1/3):
U = p(rho) - rho/3 <= 0 and psi = sqrt(2U/G), G < 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize

CS2 = 1.0 / 3.0


# --------------------------------------------------------------------------
# Equations of state
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class EOS:
    """One equation of state with its constants.

    kind: "vdw" (Eq. 21), "pr" (Eq. 29), "cs" (Carnahan-Starling) or "ideal".
    K multiplies the whole pressure (Eq. 21, Eq. 29).
    """

    kind: str
    a: float
    b: float
    R: float = 1.0
    K: float = 1.0
    omega: float = 0.344  # Peng-Robinson acentric factor (Sec. 4)

    # raw (K = 1) pressure and its first two density derivatives --------
    def _raw(self, rho, T, Tc=None):
        rho = np.asarray(rho, dtype=np.float64)
        a, b, R = self.a, self.b, self.R
        if self.kind == "ideal":
            return rho / 3.0, np.full_like(rho, 1.0 / 3.0), np.zeros_like(rho)
        if self.kind == "vdw":
            d = 1.0 - b * rho
            p = rho * R * T / d - a * rho**2
            dp = R * T / d**2 - 2.0 * a * rho
            d2p = 2.0 * R * T * b / d**3 - 2.0 * a
            return p, dp, d2p
        if self.kind == "cs":
            eta = b * rho / 4.0
            om = 1.0 - eta
            h = eta * (1.0 + eta + eta**2 - eta**3) / om**3
            h1 = (1.0 + 4.0 * eta + 4.0 * eta**2 - 4.0 * eta**3 + eta**4) / om**4
            h2 = (8.0 + 20.0 * eta - 4.0 * eta**2) / om**5
            c = 4.0 / b
            p = R * T * c * h - a * rho**2
            dp = R * T * h1 - 2.0 * a * rho
            d2p = R * T * h2 * (b / 4.0) - 2.0 * a
            return p, dp, d2p
        if self.kind == "pr":
            if Tc is None:
                raise ValueError("PR pressure needs Tc for alpha(T)")
            kap = 0.37464 + 1.54226 * self.omega - 0.26992 * self.omega**2
            alpha = (1.0 + kap * (1.0 - math.sqrt(T / Tc))) ** 2
            d = 1.0 - b * rho
            q = 1.0 + 2.0 * b * rho - b**2 * rho**2
            q1 = 2.0 * b - 2.0 * b**2 * rho
            q2 = -2.0 * b**2
            aa = a * alpha
            p = rho * R * T / d - aa * rho**2 / q
            # d/drho of rho^2/q and its second derivative
            g = rho**2 / q
            g1 = (2.0 * rho * q - rho**2 * q1) / q**2
            g2 = (2.0 * q - rho**2 * q2) / q**2 - 2.0 * q1 * (2.0 * rho * q - rho**2 * q1) / q**3
            dp = R * T / d**2 - aa * g1
            d2p = 2.0 * R * T * b / d**3 - aa * g2
            del g
            return p, dp, d2p
        raise ValueError(f"unknown EOS kind {self.kind!r}")

    def p(self, rho, T, Tc=None):
        """Pressure K*p_EOS(rho; T)."""
        return self.K * self._raw(rho, T, Tc)[0]

    def dp(self, rho, T, Tc=None):
        return self.K * self._raw(rho, T, Tc)[1]

    def d2p(self, rho, T, Tc=None):
        return self.K * self._raw(rho, T, Tc)[2]


def vdw(K: float = 0.3) -> EOS:
    """Sec. 3, Eq. (21): a = 9/49, b = 2/21, R = 1."""
    return EOS("vdw", 9.0 / 49.0, 2.0 / 21.0, 1.0, K)


def carnahan_starling(K: float = 1.0) -> EOS:
    """Carnahan-Starling with a = 1, b = 4, R = 1 (the workloads' EOS)."""
    return EOS("cs", 1.0, 4.0, 1.0, K)


def peng_robinson(K: float = 0.5, a: float = 2.0 / 49.0) -> EOS:
    """Sec. 4, Eq. (29): b = 2/21, R = 1, omega = 0.344; a is not printed (reading: 2/49)."""
    return EOS("pr", a, 2.0 / 21.0, 1.0, K, 0.344)


# --------------------------------------------------------------------------
# Critical point
# --------------------------------------------------------------------------
def critical_point(eos: EOS) -> tuple[float, float]:
    """(rho_c, T_c): dp/drho = 0 and d2p/drho2 = 0 (K does not change them).

    vdW has the closed form rho_c = 1/(3b), T_c = 8a/(27 b R).  Other EOS are
    solved numerically: for each T the inflection density rho*(T) is found,
    then T is adjusted until dp/drho(rho*(T)) = 0.
    """
    if eos.kind == "vdw":
        return 1.0 / (3.0 * eos.b), 8.0 * eos.a / (27.0 * eos.b * eos.R)
    if eos.kind == "ideal":
        raise ValueError("ideal gas has no critical point")
    if eos.kind == "pr":
        # alpha(Tc) = 1, so at T = Tc the PR isotherm is the a-alpha=a one.
        # Solve for (rho, T) with alpha frozen at 1.
        def res(v):
            rho, T = v
            e = EOS("pr", eos.a, eos.b, eos.R, 1.0, eos.omega)
            _, d1, d2 = e._raw(rho, T, Tc=T)
            return [d1, d2]

        sol = optimize.fsolve(res, [0.25 / eos.b, 0.17 * eos.a / (eos.b * eos.R)], xtol=1e-15)
        return float(sol[0]), float(sol[1])
    rho_hi = 0.999 * (4.0 / eos.b if eos.kind == "cs" else 1.0 / eos.b)

    def rho_star(T):
        e = EOS(eos.kind, eos.a, eos.b, eos.R, 1.0, eos.omega)
        f = lambda r: e._raw(r, T)[2]
        return optimize.brentq(f, 1e-9, rho_hi * 0.9, xtol=1e-16, rtol=1e-15, maxiter=500)

    def g(T):
        e = EOS(eos.kind, eos.a, eos.b, eos.R, 1.0, eos.omega)
        return e._raw(rho_star(T), T)[1]

    scale = eos.a / (eos.b * eos.R)
    Tc = optimize.brentq(g, 0.05 * scale, 0.9 * scale, xtol=1e-16, rtol=1e-15, maxiter=500)
    return rho_star(Tc), Tc


# --------------------------------------------------------------------------
# Spinodal and Maxwell construction
# --------------------------------------------------------------------------
def spinodal(eos: EOS, T: float, Tc: float | None = None) -> tuple[float, float]:
    """Densities where dp/drho = 0 (the mechanical-instability bounds)."""
    rc, _ = critical_point(eos)
    hi = 0.999 * (4.0 / eos.b if eos.kind == "cs" else 1.0 / eos.b)
    f = lambda r: eos._raw(r, T, Tc)[1]
    lo = optimize.brentq(f, 1e-12, rc, xtol=1e-16, rtol=1e-15)
    up = optimize.brentq(f, rc, hi, xtol=1e-16, rtol=1e-15)
    return lo, up


def maxwell(eos: EOS, T: float, Tc: float | None = None) -> tuple[float, float]:
    """Coexisting (rho_v, rho_l): equal pressure and equal area in the specific volume.

    For a trial pressure P between the spinodal pressures, rho_v(P) and rho_l(P)
    are the outer roots of p(rho) = P, and the equal-area rule reads
    A(P) = int_{1/rho_l}^{1/rho_v} (p(1/v) - P) dv = 0.  A(P) falls
    monotonically with P, so the saturation pressure is a bracketed 1-D root.
    """
    s_lo, s_hi = spinodal(eos, T, Tc)
    p = lambda r: float(eos._raw(r, T, Tc)[0])
    rho_hi = 0.999 * (4.0 / eos.b if eos.kind == "cs" else 1.0 / eos.b)
    p_top = p(s_lo)                      # local maximum of the loop
    p_bot = max(p(s_hi), 1e-12 * p_top)  # local minimum (the vapour needs p > 0)

    def roots(P):
        rv = optimize.brentq(lambda r: p(r) - P, 1e-300 if P > 0 else 1e-12, s_lo, xtol=1e-300, rtol=1e-15, maxiter=500)
        rl = optimize.brentq(lambda r: p(r) - P, s_hi, rho_hi, xtol=1e-300, rtol=1e-15, maxiter=500)
        return rv, rl

    def area(P):
        # in the specific volume v = 1/rho the integrand p(1/v) - P is bounded
        rv, rl = roots(P)
        vv, vl = 1.0 / rv, 1.0 / rl
        return integrate.quad(lambda v: p(1.0 / v) - P, vl, vv, points=[1.0 / s_hi, 1.0 / s_lo],
                              epsabs=1e-13 * P * (vv - vl), epsrel=1e-13, limit=400)[0]

    lo, hi = p_bot * (1 + 1e-12), p_top * (1 - 1e-12)
    if not (area(lo) > 0 > area(hi)):
        raise RuntimeError("Maxwell construction: no equal-area pressure between the spinodals")
    P = optimize.brentq(area, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=500)
    rv, rl = roots(P)
    return float(rv), float(rl)


# --------------------------------------------------------------------------
# Pseudo-potential fields
# --------------------------------------------------------------------------
def U_of_rho(eos: EOS, rho, T, Tc=None):
    """Eq. (10): U = p - c_s^2 rho."""
    return eos.p(rho, T, Tc) - CS2 * np.asarray(rho, dtype=np.float64)


def psi_of_rho(eos: EOS, rho, T, G=-1.0, Tc=None):
    """psi = sqrt(2U/G) (Eq. 10 with U = G psi^2 / 2)."""
    return np.sqrt(np.maximum(0.0, 2.0 * U_of_rho(eos, rho, T, Tc) / G))


# --------------------------------------------------------------------------
# Mechanical stability condition, Eq. (17)
# --------------------------------------------------------------------------
def mechanical_stability(eos: EOS, T: float, A: float, G: float = -1.0, Tc=None,
                         guess: tuple[float, float] | None = None) -> tuple[float, float]:
    """(rho_v, rho_l) from Eq. (17) with eps = -2A.

    Conditions: p(rho_v) = p(rho_l) = p_c and
        int_{rho_v}^{rho_l} (p_c - p(rho)) psi'(rho) / psi^(1+eps) drho = 0.
    """
    eps = -2.0 * A
    p = lambda r: float(eos._raw(r, T, Tc)[0]) * eos.K
    psi = lambda r: math.sqrt(max(0.0, 2.0 * (p(r) - r / 3.0) / G))
    dpsi = lambda r: (float(eos._raw(r, T, Tc)[1]) * eos.K - 1.0 / 3.0) / (G * psi(r))

    def res(v):
        rv, rl = v
        pc = p(rv)
        val = integrate.quad(lambda r: (pc - p(r)) * dpsi(r) / psi(r) ** (1.0 + eps), rv, rl,
                             epsabs=1e-15, epsrel=1e-12, limit=400)[0]
        return [p(rl) - pc, val]

    if guess is None:
        guess = maxwell(eos, T, Tc)
    sol, info, ier, msg = optimize.fsolve(res, list(guess), xtol=1e-13, full_output=True)
    r = res(sol)
    if ier != 1 and max(abs(r[0]), abs(r[1])) > 1e-12:
        raise RuntimeError(f"Eq.(17) solve failed: {msg}")
    return float(sol[0]), float(sol[1])


# --------------------------------------------------------------------------
# Leading-order surface tension, Eqs. (14), (20), (28)
# --------------------------------------------------------------------------
def sigma_leading_order(eos: EOS, T: float, A: float, kappa: float = 0.0, G: float = -1.0,
                        Tc=None, n: int = 200001) -> float:
    """sigma = (A-1)(G/6) int (dpsi/dn)^2 dn * (1 - kappa).

    From P_xx = p_c (Eq. 14 with a = 3A, b = 3):  (G/4)(A psi'^2 + psi psi'') = p_c - p_0,
    so y = psi'^2 satisfies  (y psi^{2A})' = (8/G) psi^{2A-1} (p_c - p_0)  and
    int psi'^2 dn = int sqrt(y) dpsi.  The coexistence densities are the Eq. (17) ones.
    """
    rv, rl = mechanical_stability(eos, T, A, G, Tc)
    r = np.linspace(rv, rl, n)
    p = eos.p(r, T, Tc)
    pc = float(p[0])
    psi = np.sqrt(np.maximum(0.0, 2.0 * (p - r / 3.0) / G))
    dpsi = (eos.dp(r, T, Tc) - 1.0 / 3.0) / (G * psi)
    integrand = psi ** (2.0 * A - 1.0) * (pc - p) * dpsi
    inner = integrate.cumulative_trapezoid(integrand, r, initial=0.0)
    y = (8.0 / G) * inner / psi ** (2.0 * A)
    y = np.maximum(y, 0.0)
    s = integrate.trapezoid(np.sqrt(y) * dpsi, r)
    return float((A - 1.0) * (G / 6.0) * s * (1.0 - kappa))


# --------------------------------------------------------------------------
# Exact discrete balance of a flat interface (s_e = s_nu = 1)
# --------------------------------------------------------------------------
def flat_force_1d(eos: EOS, rho: np.ndarray, T: float, A: float, G: float = -1.0, Tc=None):
    """Eq. (9) for a field that depends on x only: the e_x = +1 weights sum to 1/2."""
    U = U_of_rho(eos, rho, T, Tc)
    psi = np.sqrt(np.maximum(0.0, 2.0 * U / G))
    Up, Um = np.roll(U, -1), np.roll(U, 1)
    pp, pm = np.roll(psi, -1), np.roll(psi, 1)
    return -(A / 2.0) * (Up - Um) - (1.0 - A) * (G / 2.0) * psi * (pp - pm)


def discrete_flat_balance(eos: EOS, T: float, A: float, N: int = 100, G: float = -1.0, Tc=None,
                          rho0: np.ndarray | None = None, width: float = 5.0):
    """Solve the steady 1-D balance of the lattice model on a periodic line of N cells.

    Unknowns rho(0..N-1); equations rho(x+1) - rho(x) - 1.5[F(x) + F(x+1)] = 0
    (one is redundant since sum F = 0) plus fixed total mass.  Returns the field
    and (rho_v, rho_l) read at the slab's centre lines.
    """
    if rho0 is None:
        rv, rl = maxwell(eos, T, Tc)
        x = np.arange(N) + 0.5
        c1, c2 = N / 4.0, 3.0 * N / 4.0
        rho0 = rv + 0.5 * (rl - rv) * (np.tanh(2 * (x - c1) / width) - np.tanh(2 * (x - c2) / width))
    mass = float(np.sum(rho0))

    def res(r):
        F = flat_force_1d(eos, r, T, A, G, Tc)
        d = np.roll(r, -1) - r - 1.5 * (F + np.roll(F, -1))
        d[-1] = (np.sum(r) - mass) / N
        return d

    sol = optimize.least_squares(res, rho0, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm",
                                 max_nfev=20000)
    r = sol.x
    if np.max(np.abs(res(r))) > 1e-11:
        raise RuntimeError(f"discrete balance did not converge: residual {np.max(np.abs(res(r)))}")
    return r, float(np.min(r)), float(np.max(r))
