"""FP64 CPU oracle of the pseudo-potential MRT lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  The product path never imports this package: only
``tests/``, the entry point's ``smoke()`` and the CPU-baseline leg of
``bench.py`` may load it.  It shares no code with the GPU library.

* ``lbm_oracle.c``  -- one time step written out in plain loops (Eqs. 1-10,
  23, 25, 26); built into ``liboracle.so`` by :func:`build`.
* ``thermo``        -- critical point, Maxwell construction, Eq. (17),
  leading-order surface tension (Eqs. 14, 20, 28) and the exact discrete
  flat-interface balance.
* ``mlp``           -- FP64 forward/backward of the surrogate network.
* :func:`laplace_fit` -- the Laplace law (Eq. 22) fitted over several drops.

A physical configuration is a plain dict with keys
``nx, ny, eos ('ideal'|'cs'|'vdw'|'pr'), a, b, R, omega_pr, K, T_over_Tc, A,
kappa, G, s_e, s_eps, s_q, s_nu, nu_gas, nu_liquid, rho_gas, rho_liquid``.  Missing keys take the defaults in
:data:`DEFAULTS`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import thermo

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EOS_CODE = {"ideal": 0, "cs": 1, "vdw": 2, "pr": 3}
EOS_CONSTANTS = {
    "ideal": dict(a=0.0, b=0.0, R=1.0),
    "cs": dict(a=1.0, b=4.0, R=1.0),
    "vdw": dict(a=9.0 / 49.0, b=2.0 / 21.0, R=1.0),
    "pr": dict(a=2.0 / 49.0, b=2.0 / 21.0, R=1.0),
}
DEFAULTS = dict(eos="cs", K=1.0, T_over_Tc=0.8, A=-0.5, kappa=0.0, G=-1.0, omega_pr=0.344,
                s_e=1.0, s_eps=1.0, s_q=8.0 / 7.0, s_nu=1.0, nu_gas=0.0, nu_liquid=0.0,
                rho_gas=0.0, rho_liquid=0.0)

# lattice velocities, used only to move between storage orders
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("eos", ctypes.c_int32),
                ("nthreads", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
                ("omega_pr", ctypes.c_double), ("K", ctypes.c_double),
                ("T", ctypes.c_double), ("Tc", ctypes.c_double),
                ("A", ctypes.c_double), ("kappa", ctypes.c_double), ("G", ctypes.c_double),
                ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
                ("s_j", ctypes.c_double), ("s_q", ctypes.c_double), ("s_nu", ctypes.c_double),
                ("nu_gas", ctypes.c_double), ("nu_liquid", ctypes.c_double),
                ("rho_gas", ctypes.c_double), ("rho_liquid", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_pressure.argtypes = [P, ctypes.c_double]
        lib.orc_pressure.restype = ctypes.c_double
        lib.orc_moment_matrix.argtypes = [dp, dp]
        lib.orc_collide_cell.argtypes = [P, dp] + [ctypes.c_double] * 5 + [dp]
        lib.orc_step.argtypes = [P, dp, dp, dp, i64p, i64p]
        lib.orc_run.argtypes = [P, dp, ctypes.c_int64, dp, i64p, i64p]
        lib.orc_init_equilibrium.argtypes = [P, dp, dp, dp, dp]
        lib.orc_interaction.argtypes = [P, dp] + [dp] * 7
        lib.orc_fields.argtypes = [P, dp, dp, dp, dp, dp, dp]
        lib.orc_observables.argtypes = [P, dp, dp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def full_config(cfg: dict) -> dict:
    """Fill defaults and EOS constants into a configuration dict."""
    c = dict(DEFAULTS)
    c.update(cfg)
    for k, v in EOS_CONSTANTS[c["eos"]].items():
        c.setdefault(k, v)
    return c


def temperature(cfg: dict) -> tuple[float, float]:
    """(T, Tc) of a configuration from thermo's critical point."""
    c = full_config(cfg)
    if c["eos"] == "ideal":
        return 0.0, 1.0
    e = thermo.EOS(c["eos"], c["a"], c["b"], c["R"], c["K"], c["omega_pr"])
    _, Tc = thermo.critical_point(e)
    return c["T_over_Tc"] * Tc, Tc


def eos_of(cfg: dict) -> thermo.EOS:
    c = full_config(cfg)
    return thermo.EOS(c["eos"], c["a"], c["b"], c["R"], c["K"], c["omega_pr"])


class Oracle:
    """One periodic lattice evolved by the FP64 oracle.  State is cell-major f[y, x, a]."""

    def __init__(self, cfg: dict, nthreads: int = 1):
        self.lib = _load()
        c = full_config(cfg)
        self.cfg = c
        T, Tc = temperature(c)
        self.T, self.Tc = T, Tc
        self.nx, self.ny = int(c["nx"]), int(c["ny"])
        self.p = _Params(self.nx, self.ny, EOS_CODE[c["eos"]], int(nthreads),
                         c["a"], c["b"], c["R"], c["omega_pr"], c["K"], T, Tc,
                         c["A"], c["kappa"], c["G"],
                         1.0, c["s_e"], c["s_eps"], 1.0, c["s_q"], c["s_nu"],
                         c["nu_gas"], c["nu_liquid"], c["rho_gas"], c["rho_liquid"])
        self.f = np.zeros((self.ny, self.nx, 9))
        self.steps = 0
        self.n_domain = 0
        self.n_bad = 0

    @property
    def nthreads(self) -> int:
        return self.p.nthreads

    @nthreads.setter
    def nthreads(self, n: int):
        self.p.nthreads = int(n)

    # -- state ----------------------------------------------------------
    def init_field(self, rho, ux=None, uy=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ny, self.nx)
        ux = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64).reshape(rho.shape)
        uy = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64).reshape(rho.shape)
        null = ctypes.POINTER(ctypes.c_double)()
        self.lib.orc_init_equilibrium(ctypes.byref(self.p), _ptr(rho),
                                      _ptr(ux) if ux is not None else null,
                                      _ptr(uy) if uy is not None else null, _ptr(self.f))
        self.steps = 0

    def set_f_soa(self, f_soa):
        """Set the state from a [9, ny, nx] array."""
        self.f = np.ascontiguousarray(np.moveaxis(np.asarray(f_soa, dtype=np.float64), 0, -1))

    def f_soa(self) -> np.ndarray:
        """The state as a [9, ny, nx] array."""
        return np.ascontiguousarray(np.moveaxis(self.f, -1, 0))

    # -- time stepping --------------------------------------------------
    def run(self, nsteps: int):
        n = self.nx * self.ny
        scratch = np.empty(12 * n)
        nd, nb = ctypes.c_int64(0), ctypes.c_int64(0)
        self.lib.orc_run(ctypes.byref(self.p), _ptr(self.f), int(nsteps), _ptr(scratch),
                         ctypes.byref(nd), ctypes.byref(nb))
        self.steps += int(nsteps)
        self.n_domain += nd.value
        self.n_bad += nb.value
        return self

    # -- read-out -------------------------------------------------------
    def fields(self) -> dict:
        shp = (self.ny, self.nx)
        out = {k: np.empty(shp) for k in ("rho", "ux", "uy", "Fx", "Fy")}
        self.lib.orc_fields(ctypes.byref(self.p), _ptr(self.f), *(_ptr(out[k]) for k in
                                                                  ("rho", "ux", "uy", "Fx", "Fy")))
        return out

    def observables(self) -> dict:
        o = np.empty(15)
        self.lib.orc_observables(ctypes.byref(self.p), _ptr(self.f), _ptr(o))
        keys = ("mass", "mom_x", "mom_y", "rho_min", "rho_max", "rho_in", "rho_out", "p_in",
                "p_out", "dp", "R_e", "sigma", "max_u", "n_domain", "n_nonfinite")
        return dict(zip(keys, (float(v) for v in o)))

    def interaction(self, rho) -> dict:
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ny, self.nx)
        keys = ("U", "psi", "Fx", "Fy", "Qxx", "Qyy", "Qxy")
        out = {k: np.empty_like(rho) for k in keys}
        self.lib.orc_interaction(ctypes.byref(self.p), _ptr(rho), *(_ptr(out[k]) for k in keys))
        return out

    def pressure(self, rho: float) -> float:
        return float(self.lib.orc_pressure(ctypes.byref(self.p), float(rho)))

    def collide_cell(self, f9, F=(0.0, 0.0), Q=(0.0, 0.0, 0.0)) -> np.ndarray:
        f9 = np.ascontiguousarray(f9, dtype=np.float64)
        out = np.empty(9)
        self.lib.orc_collide_cell(ctypes.byref(self.p), _ptr(f9), float(F[0]), float(F[1]),
                                  float(Q[0]), float(Q[1]), float(Q[2]), _ptr(out))
        return out


def moment_matrix() -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    M, Minv = np.empty(81), np.empty(81)
    lib.orc_moment_matrix(_ptr(M), _ptr(Minv))
    return M.reshape(9, 9), Minv.reshape(9, 9)


def laplace_fit(dp, R) -> tuple[float, float]:
    """Eq. (22), as tested over drop sizes in Sec. 3.1.1 and Sec. 4.1: dp = sigma / R.
    sigma is the least-squares fit of that line through the origin, i.e. the sigma
    minimising sum_i (dp_i - sigma x_i)^2 with x_i = 1 / R_i, whose normal equation
    gives sigma = sum_i dp_i x_i / sum_i x_i^2.  Also returns how far the drops are
    from one sigma: (max - min) / |mean| of dp_i R_i."""
    dp = [float(v) for v in dp]
    R = [float(v) for v in R]
    if not dp or len(dp) != len(R) or any(not r > 0.0 for r in R):
        raise ValueError("laplace_fit needs as many positive radii as pressure jumps (at least one)")
    num = den = 0.0
    for d, r in zip(dp, R):
        x = 1.0 / r
        num += d * x
        den += x * x
    each = [d * r for d, r in zip(dp, R)]
    mean = sum(each) / len(each)
    return num / den, (max(each) - min(each)) / abs(mean)
