"""ctypes binding of liblbm's C ABI (include/lbm.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  PyTorch provides the device memory (the two distribution buffers are
torch tensors handed to ``lbm_create_ext``) and the stream (torch's current
stream by default).  There is no fallback: if ``liblbm.so`` is missing or no
HIP device is present, constructing a :class:`Lattice` raises.

Parameters are passed as a plain dict with keys ``nx, ny, eos ('ideal'|'cs'|
'vdw'|'pr'), a, b, R, omega_pr, K, T_over_Tc, A, kappa, G, s_e, s_eps, s_q,
s_nu, nu_gas, nu_liquid, rho_gas, rho_liquid, precision ('fp64'|'fp32')``;
missing keys take :data:`DEFAULTS`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")
Q = 9  # LBM_Q of include/lbm.h: element (a, y, x) of a state buffer at (Q * y + a) * pitch + x

EOS = {"ideal": 0, "cs": 1, "vdw": 2, "pr": 3}
EOS_CONSTANTS = {
    "ideal": dict(a=1.0, b=1.0, R=1.0),
    "cs": dict(a=1.0, b=4.0, R=1.0),
    "vdw": dict(a=9.0 / 49.0, b=2.0 / 21.0, R=1.0),
    "pr": dict(a=2.0 / 49.0, b=2.0 / 21.0, R=1.0),
}
PRECISION = {"fp64": 0, "fp32": 1}
FIELDS = {"rho": 0, "ux": 1, "uy": 2, **{f"f{a}": 3 + a for a in range(9)}}
DEFAULTS = dict(eos="cs", K=1.0, T_over_Tc=0.8, A=-0.5, kappa=0.0, G=-1.0, omega_pr=0.344,
                s_e=1.0, s_eps=1.0, s_q=8.0 / 7.0, s_nu=1.0, nu_gas=0.0, nu_liquid=0.0,
                rho_gas=0.0, rho_liquid=0.0, precision="fp64")

STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
          -4: "LBM_ENONFINITE", -5: "LBM_EDOMAIN", -6: "LBM_ESTATE"}


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("eos", ctypes.c_int32),
                ("precision", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
                ("omega_pr", ctypes.c_double), ("K", ctypes.c_double),
                ("T_over_Tc", ctypes.c_double), ("A", ctypes.c_double),
                ("kappa", ctypes.c_double), ("G", ctypes.c_double),
                ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
                ("s_nu", ctypes.c_double), ("nu_gas", ctypes.c_double),
                ("nu_liquid", ctypes.c_double), ("rho_gas", ctypes.c_double),
                ("rho_liquid", ctypes.c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64)] + [
        (k, ctypes.c_double) for k in ("mass", "mom_x", "mom_y", "rho_min", "rho_max", "rho_in",
                                       "rho_out", "p_in", "p_out", "dp", "R_e", "sigma", "max_u")
    ] + [("n_nonfinite", ctypes.c_int64), ("n_domain", ctypes.c_int64)]


class Launch(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("steps_per_pass", ctypes.c_int32)]


class BatchLaunch(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("spin_limit", ctypes.c_int64), ("force_spin_limit", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("ntiles", ctypes.c_int32),
                ("resident_per_cu", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32)]


BATCH_MODES = {"persistent": 0, "per_step": 1}


_lib = None


def load_library(path: str | None = None):
    """Load liblbm.so (``LIB_PATH`` unless given) and declare its entry points.
    Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is not built (python -m paper_1412_7228_amd.build)")
    # torch first: the library must bind to the HIP runtime that torch loads (its
    # buffers and streams are torch's); loaded first, the library would pull in a
    # second HIP/HSA runtime that cannot open the device
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    P = ctypes.POINTER(Params)
    st = ctypes.c_int
    decl = {
        "lbm_params_default": (st, [P]),
        "lbm_critical_temperature": (st, [P, dp]),
        "lbm_coexistence": (st, [P, dp, dp]),
        "lbm_laplace_fit": (st, [dp, dp, ctypes.c_int32, dp, dp]),
        "lbm_buffer_bytes": (ctypes.c_size_t, [P]),
        "lbm_create": (st, [P, vp, ctypes.POINTER(vp)]),
        "lbm_create_ext": (st, [P, vp, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]),
        "lbm_destroy": (None, [vp]),
        "lbm_set_launch": (st, [vp, ctypes.POINTER(Launch)]),
        "lbm_get_launch": (st, [vp, ctypes.POINTER(Launch)]),
        "lbm_init_field": (st, [vp, dp, dp, dp]),
        "lbm_set_distributions": (st, [vp, dp]),
        "lbm_step": (st, [vp, ctypes.c_int64]),
        "lbm_step_rows": (st, [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "lbm_observables": (st, [vp, ctypes.POINTER(Obs)]),
        "lbm_observables_noalloc": (st, [vp, ctypes.POINTER(Obs)]),
        "lbm_noalloc_max_cells": (ctypes.c_int64, []),
        "lbm_get_field": (st, [vp, ctypes.c_int32, dp]),
        "lbm_save_state": (st, [vp, vp, ctypes.POINTER(ctypes.c_size_t)]),
        "lbm_load_state": (st, [vp, vp, ctypes.c_size_t]),
        "lbm_sync": (st, [vp]),
        "lbm_state_info": (st, [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(vp),
                                ctypes.POINTER(ctypes.c_int32)]),
        "lbm_batch_create": (st, [P, ctypes.c_int32, vp, ctypes.POINTER(vp)]),
        "lbm_batch_destroy": (None, [vp]),
        "lbm_batch_set_launch": (st, [vp, ctypes.POINTER(BatchLaunch)]),
        "lbm_batch_get_launch": (st, [vp, ctypes.POINTER(BatchLaunch)]),
        "lbm_batch_init_field": (st, [vp, ctypes.c_int32, dp, dp, dp]),
        "lbm_batch_step": (st, [vp, ctypes.c_int64]),
        "lbm_batch_sync": (st, [vp]),
        "lbm_batch_observables": (st, [vp, ctypes.POINTER(Obs)]),
        "lbm_batch_get_field": (st, [vp, ctypes.c_int32, ctypes.c_int32, dp]),
        "lbm_mlp_param_count": (ctypes.c_int32, []),
        "lbm_mlp_create": (st, [ctypes.c_int32, vp, ctypes.POINTER(vp)]),
        "lbm_mlp_destroy": (None, [vp]),
        "lbm_mlp_set_params": (st, [vp, fp]),
        "lbm_mlp_get_params": (st, [vp, fp]),
        "lbm_mlp_forward": (st, [vp, fp, ctypes.c_int32, fp]),
        "lbm_mlp_backward": (st, [vp, fp, fp, ctypes.c_int32, fp, fp]),
        "lbm_mlp_set_data": (st, [vp, fp, fp, ctypes.c_int32]),
        "lbm_mlp_train": (st, [vp, ctypes.c_int32, ctypes.c_float, fp]),
        "lbm_strerror": (ctypes.c_char_p, [st]),
        "lbm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in decl.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise LBMError(status, load_library().lbm_last_error().decode())


def make_params(cfg: dict) -> Params:
    c = dict(DEFAULTS)
    c.update(cfg)
    for k, v in EOS_CONSTANTS[c["eos"]].items():
        c.setdefault(k, v)
    return Params(int(c["nx"]), int(c["ny"]), EOS[c["eos"]], PRECISION[c["precision"]],
                  float(c["a"]), float(c["b"]), float(c["R"]), float(c["omega_pr"]),
                  float(c["K"]), float(c["T_over_Tc"]), float(c["A"]), float(c["kappa"]),
                  float(c["G"]), float(c["s_e"]), float(c["s_eps"]), float(c["s_q"]),
                  float(c["s_nu"]), float(c["nu_gas"]), float(c["nu_liquid"]),
                  float(c["rho_gas"]), float(c["rho_liquid"]))


def critical_temperature(cfg: dict) -> float:
    lib = load_library()
    p = make_params(dict(cfg, nx=cfg.get("nx", 3), ny=cfg.get("ny", 3)))
    tc = ctypes.c_double()
    _check(lib.lbm_critical_temperature(ctypes.byref(p), ctypes.byref(tc)))
    return tc.value


def coexistence(cfg: dict) -> tuple[float, float]:
    """Maxwell (rho_v, rho_l) of the configuration's EOS at its T/Tc (host computation)."""
    lib = load_library()
    p = make_params(dict(cfg, nx=cfg.get("nx", 3), ny=cfg.get("ny", 3)))
    rv, rl = ctypes.c_double(), ctypes.c_double()
    _check(lib.lbm_coexistence(ctypes.byref(p), ctypes.byref(rv), ctypes.byref(rl)))
    return rv.value, rl.value


def laplace_fit(dp, R_e) -> tuple[float, float]:
    """Laplace law over drops (lbm_laplace_fit): sigma as the least-squares slope of dp
    against 1/R_e through the origin, and the relative spread of dp * R_e."""
    lib = load_library()
    d = np.ascontiguousarray(dp, dtype=np.float64).ravel()
    r = np.ascontiguousarray(R_e, dtype=np.float64).ravel()
    if d.size != r.size:
        raise ValueError("dp and R_e differ in length")
    sig, spread = ctypes.c_double(), ctypes.c_double()
    _check(lib.lbm_laplace_fit(_dptr(d), _dptr(r), int(d.size), ctypes.byref(sig), ctypes.byref(spread)))
    return sig.value, spread.value


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Lattice:
    """One periodic lattice on the current HIP device.

    ``stream``: a ``torch.cuda.Stream`` (default: torch's current stream).
    ``torch_buffers``: allocate the two distribution buffers with torch
    (default) or let the library ``hipMalloc`` them.
    """

    def __init__(self, cfg: dict, stream=None, torch_buffers: bool = True):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP device; none is visible")
        self.lib = load_library()
        self.cfg = dict(DEFAULTS, **cfg)
        self.p = make_params(cfg)
        self.nx, self.ny = self.p.nx, self.p.ny
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        self._bufs = None
        if torch_buffers:
            nbytes = self.lib.lbm_buffer_bytes(ctypes.byref(self.p))
            if nbytes == 0:
                _check(self.lib.lbm_create(ctypes.byref(self.p), sp, ctypes.byref(h)))
            self._bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
            _check(self.lib.lbm_create_ext(ctypes.byref(self.p), sp,
                                           ctypes.c_void_p(self._bufs[0].data_ptr()),
                                           ctypes.c_void_p(self._bufs[1].data_ptr()),
                                           nbytes, ctypes.byref(h)))
        else:
            _check(self.lib.lbm_create(ctypes.byref(self.p), sp, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- launch shape --------------------------------------------------------
    @property
    def launch(self) -> tuple[int, int, int]:
        """(tile_x, tile_y, steps_per_pass) of the step launches."""
        l = Launch()
        _check(self.lib.lbm_get_launch(self.h, ctypes.byref(l)))
        return l.tile_x, l.tile_y, l.steps_per_pass

    def set_launch(self, tile_x: int = 0, tile_y: int = 0, steps_per_pass: int = 0):
        l = Launch(int(tile_x), int(tile_y), int(steps_per_pass))
        _check(self.lib.lbm_set_launch(self.h, ctypes.byref(l)))

    # -- state ---------------------------------------------------------------
    def init_field(self, rho, ux=None, uy=None):
        shp = (self.ny, self.nx)
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(shp)
        u = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64).reshape(shp)
        v = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64).reshape(shp)
        null = ctypes.POINTER(ctypes.c_double)()
        _check(self.lib.lbm_init_field(self.h, _dptr(r), _dptr(u) if u is not None else null,
                                       _dptr(v) if v is not None else null))

    def set_distributions(self, f_soa):
        f = np.ascontiguousarray(f_soa, dtype=np.float64).reshape(9, self.ny, self.nx)
        _check(self.lib.lbm_set_distributions(self.h, _dptr(f)))

    def step(self, n: int = 1):
        _check(self.lib.lbm_step(self.h, int(n)))
        return self

    def step_rows(self, n: int, y_begin: int, rows: int, more: bool = False):
        """One launch of n (1 or 2) steps that updates only rows [y_begin, y_begin + rows);
        ``more``: further ranges of the same steps follow (the source stays current)."""
        _check(self.lib.lbm_step_rows(self.h, int(n), int(y_begin), int(rows), 1 if more else 0))
        return self

    def sync(self):
        _check(self.lib.lbm_sync(self.h))

    # -- read-out ------------------------------------------------------------
    def observables(self, check: bool = True, noalloc: bool = False) -> dict:
        """FP64 observables (lbm_observables; ``noalloc``: lbm_observables_noalloc, the
        variant that allocates nothing)."""
        o = Obs()
        fn = self.lib.lbm_observables_noalloc if noalloc else self.lib.lbm_observables
        st = fn(self.h, ctypes.byref(o))
        if check:
            _check(st)
        d = {k: getattr(o, k) for k, _ in Obs._fields_}
        d["status"] = st
        return d

    def field(self, name: str) -> np.ndarray:
        out = np.empty((self.ny, self.nx))
        _check(self.lib.lbm_get_field(self.h, FIELDS[name], _dptr(out)))
        return out

    def f_soa(self) -> np.ndarray:
        return np.stack([self.field(f"f{a}") for a in range(9)])

    def fields(self) -> dict:
        return {k: self.field(k) for k in ("rho", "ux", "uy")}

    def save_state(self) -> bytes:
        n = ctypes.c_size_t(0)
        _check(self.lib.lbm_save_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self.lib.lbm_save_state(self.h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self.lib.lbm_load_state(self.h, buf, len(blob)))

    def state_tensor(self):
        """The current device state as a torch view [9, ny, pitch] over the library's
        row-interleaved layout (plane stride pitch, row stride 9 * pitch; post-collision
        values before streaming), in the working precision.
        Valid until the next step; writes to it change the state."""
        import torch

        if self._bufs is None:
            raise RuntimeError("state_tensor needs torch-allocated buffers")
        ptr = self.info()["f_cur"]
        buf = next(b for b in self._bufs if b.data_ptr() == ptr)
        dt = torch.float32 if self.p.precision == PRECISION["fp32"] else torch.float64
        pitch = (self.nx + 63) // 64 * 64
        return buf.view(dt).as_strided((Q, self.ny, pitch), (pitch, Q * pitch, 1))

    def info(self) -> dict:
        step, ptr, pitch = ctypes.c_int64(), ctypes.c_void_p(), ctypes.c_int32()
        _check(self.lib.lbm_state_info(self.h, ctypes.byref(step), ctypes.byref(ptr),
                                       ctypes.byref(pitch)))
        return dict(step=step.value, f_cur=ptr.value, pitch=pitch.value)


class Batch:
    """Many independent lattices advanced together (``lbm_batch_*``).

    ``cfgs``: one parameter dict per domain (same EOS kind and precision).
    """

    def __init__(self, cfgs: list, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP device; none is visible")
        self.lib = load_library()
        self.cfgs = [dict(DEFAULTS, **c) for c in cfgs]
        arr = (Params * len(cfgs))(*[make_params(c) for c in cfgs])
        self._params = arr
        self.shapes = [(p.ny, p.nx) for p in arr]
        # a stream of its own (default priority), so the library can use HIP graphs
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        _check(self.lib.lbm_batch_create(arr, len(cfgs), ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(h)))
        self.h = h
        self.n = len(cfgs)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, mode: str = "per_step", tile_x: int = 0, tile_y: int = 0,
                   spin_limit: int = 0, force_spin_limit: bool = False, steps_per_pass: int = 0):
        l = BatchLaunch(BATCH_MODES[mode], int(tile_x), int(tile_y), int(spin_limit),
                        int(force_spin_limit), 0, 0, 0, int(steps_per_pass))
        _check(self.lib.lbm_batch_set_launch(self.h, ctypes.byref(l)))

    @property
    def launch(self) -> dict:
        l = BatchLaunch()
        _check(self.lib.lbm_batch_get_launch(self.h, ctypes.byref(l)))
        inv = {v: k for k, v in BATCH_MODES.items()}
        return dict(mode=inv[l.mode], tile_x=l.tile_x, tile_y=l.tile_y, spin_limit=l.spin_limit,
                    grid=l.grid, ntiles=l.ntiles, resident_per_cu=l.resident_per_cu,
                    steps_per_pass=l.steps_per_pass)

    def init_field(self, i: int, rho, ux=None, uy=None):
        shp = self.shapes[i]
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(shp)
        u = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64).reshape(shp)
        v = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64).reshape(shp)
        null = ctypes.POINTER(ctypes.c_double)()
        _check(self.lib.lbm_batch_init_field(self.h, int(i), _dptr(r),
                                             _dptr(u) if u is not None else null,
                                             _dptr(v) if v is not None else null))

    def step(self, n: int = 1):
        _check(self.lib.lbm_batch_step(self.h, int(n)))
        return self

    def sync(self):
        _check(self.lib.lbm_batch_sync(self.h))

    def observables(self, check: bool = False) -> list:
        out = (Obs * self.n)()
        st = self.lib.lbm_batch_observables(self.h, out)
        if check or st in (-1, -2, -3, -6):
            _check(st)
        return [{k: getattr(o, k) for k, _ in Obs._fields_} for o in out]

    def field(self, i: int, name: str) -> np.ndarray:
        out = np.empty(self.shapes[i])
        _check(self.lib.lbm_batch_get_field(self.h, int(i), FIELDS[name], _dptr(out)))
        return out

    def f_soa(self, i: int) -> np.ndarray:
        return np.stack([self.field(i, f"f{a}") for a in range(9)])


def _fptr(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class MLP:
    """The surrogate network of the library (``lbm_mlp_*``): 3 -> 128 -> 128 -> 128 -> 3."""

    def __init__(self, max_batch: int = 1024, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP device; none is visible")
        self.lib = load_library()
        self.nparams = int(self.lib.lbm_mlp_param_count())
        self.max_batch = int(max_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(self.lib.lbm_mlp_create(self.max_batch, ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        _check(self.lib.lbm_mlp_set_params(self.h, _fptr(p)))

    def params(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        _check(self.lib.lbm_mlp_get_params(self.h, _fptr(out)))
        return out

    def forward(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
        out = np.empty_like(x)
        for i in range(0, len(x), self.max_batch):
            xs = np.ascontiguousarray(x[i:i + self.max_batch])
            ys = np.empty_like(xs)
            _check(self.lib.lbm_mlp_forward(self.h, _fptr(xs), len(xs), _fptr(ys)))
            out[i:i + len(xs)] = ys
        return out

    def backward(self, x, dy):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
        dy = np.ascontiguousarray(dy, dtype=np.float32).reshape(-1, 3)
        grad = np.empty(self.nparams, dtype=np.float32)
        dx = np.empty_like(x)
        _check(self.lib.lbm_mlp_backward(self.h, _fptr(x), _fptr(dy), len(x), _fptr(grad), _fptr(dx)))
        return grad, dx

    def set_data(self, x, t):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
        t = np.ascontiguousarray(t, dtype=np.float32).reshape(-1, 3)
        _check(self.lib.lbm_mlp_set_data(self.h, _fptr(x), _fptr(t), len(x)))

    def train(self, iters: int, lr: float) -> np.ndarray:
        loss = np.empty(max(1, iters), dtype=np.float32)
        _check(self.lib.lbm_mlp_train(self.h, int(iters), float(lr), _fptr(loss)))
        return loss[:iters]
