"""The C-ABI library without a GPU: it loads, exports every declared entry point,
validates parameters before touching the device, and its host-side critical
temperature agrees with the oracle's thermodynamics."""
import ctypes
import os
import re

import pytest

from paper_1412_7228_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1412_7228_amd import build

        build.build()
    return lbm.load_library()


def test_header_declares_the_core_entry_points():
    names = declared_symbols()
    for core in ("lbm_create", "lbm_init_field", "lbm_step", "lbm_observables"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_noalloc_limit_is_exported_without_a_device(lib):
    """The size limit of lbm_observables_noalloc is a host constant: 2^28 cells."""
    lib.lbm_noalloc_max_cells.restype = ctypes.c_int64
    assert lib.lbm_noalloc_max_cells() == 2**28


def test_defaults_and_strerror(lib):
    p = lbm.Params()
    assert lib.lbm_params_default(ctypes.byref(p)) == 0
    assert (p.nx, p.ny, p.eos, p.precision) == (64, 64, 1, 0)
    assert lib.lbm_strerror(-4) == b"non-finite or non-positive density"
    assert lib.lbm_params_default(None) == -1


@pytest.mark.parametrize("bad", [dict(nx=2), dict(ny=0), dict(s_nu=2.0), dict(s_e=0.0),
                                 dict(G=0.5), dict(precision_code=7), dict(eos_code=9),
                                 dict(K=-1.0), dict(T_over_Tc=0.0),
                                 dict(nx=65536, ny=65536)])  # one FP64 plane of 32 GiB
def test_invalid_parameters_are_rejected_before_device_use(lib, bad):
    cfg = dict(nx=16, ny=16)
    cfg.update({k: v for k, v in bad.items() if not k.endswith("_code")})
    p = lbm.make_params(cfg)
    if "precision_code" in bad:
        p.precision = bad["precision_code"]
    if "eos_code" in bad:
        p.eos = bad["eos_code"]
    h = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert not h.value
    assert lib.lbm_last_error() != b""
    assert lib.lbm_buffer_bytes(ctypes.byref(p)) == 0


def test_buffer_bytes_pitch(lib):
    """ny lattice rows, each the rows of the 9 planes back to back, pitch elements
    each (nx rounded up to 64); the binding's constant is the header's."""
    m = re.search(r"#define\s+LBM_Q\s+(\d+)", open(os.path.join(ROOT, "include", "lbm.h")).read())
    assert m and int(m.group(1)) == lbm.Q == 9
    p = lbm.make_params(dict(nx=100, ny=7, precision="fp32"))
    assert lib.lbm_buffer_bytes(ctypes.byref(p)) == 7 * 9 * 128 * 4
    p = lbm.make_params(dict(nx=128, ny=3))
    assert lib.lbm_buffer_bytes(ctypes.byref(p)) == 3 * 9 * 128 * 8


@pytest.mark.parametrize("eos", ["cs", "vdw", "pr"])
def test_library_critical_temperature_matches_oracle(lib, oracle_mod, eos):
    tc_lib = lbm.critical_temperature(dict(eos=eos))
    _, tc_orc = oracle_mod.temperature(dict(eos=eos, T_over_Tc=1.0))
    assert abs(tc_lib / tc_orc - 1) < 1e-13


def test_critical_temperature_rejects_ideal(lib):
    with pytest.raises(lbm.LBMError):
        lbm.critical_temperature(dict(eos="ideal"))


@pytest.mark.parametrize("eos,tr", [("cs", 0.8), ("cs", 0.6), ("cs", 0.85), ("cs", 0.7), ("vdw", 0.9),
                                    ("vdw", 0.7), ("vdw", 0.76), ("vdw", 0.82), ("pr", 0.8), ("pr", 0.9)])
def test_library_coexistence_matches_oracle_maxwell(lib, oracle_mod, eos, tr):
    from oracle import thermo as th

    cfg = dict(eos=eos, T_over_Tc=tr)
    rv, rl = lbm.coexistence(cfg)
    T, Tc = oracle_mod.temperature(cfg)
    ov, ol = th.maxwell(oracle_mod.eos_of(cfg), T, Tc)
    assert abs(rv / ov - 1) < 1e-9 and abs(rl / ol - 1) < 1e-9


def test_coexistence_rejects_supercritical(lib):
    with pytest.raises(lbm.LBMError):
        lbm.coexistence(dict(eos="cs", T_over_Tc=1.05))


@pytest.mark.parametrize("offset,nbytes", [(8, None), (0, 16)])
def test_caller_buffers_misaligned_or_short_are_rejected(lib, offset, nbytes):
    """lbm_create_ext checks the caller's buffers before any device call: a
    pointer that is not 256-byte aligned, or a size below lbm_buffer_bytes, is
    LBM_EINVAL and the error text names the bytes needed."""
    p = lbm.make_params(dict(nx=16, ny=16))
    need = lib.lbm_buffer_bytes(ctypes.byref(p))
    host = (ctypes.c_char * (2 * need + 1024))()
    base = (ctypes.addressof(host) + 255) // 256 * 256
    a, b = base + offset, base + need + 256
    h = ctypes.c_void_p()
    rc = lib.lbm_create_ext(ctypes.byref(p), None, ctypes.c_void_p(a), ctypes.c_void_p(b),
                            need if nbytes is None else nbytes, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert str(need).encode() in lib.lbm_last_error()


def test_largest_plane_is_accepted_and_one_more_row_is_not(lib):
    """One plane's worth of elements (ny * pitch) must stay below 4 GiB (it bounds the
    cell count): an FP32 32768 x 32767 lattice (4,294,836,224 bytes a plane) is valid,
    32768 x 32768 is not."""
    ok = lbm.make_params(dict(nx=32768, ny=32767, precision="fp32"))
    assert lib.lbm_buffer_bytes(ctypes.byref(ok)) == 9 * 32767 * 32768 * 4
    bad = lbm.make_params(dict(nx=32768, ny=32768, precision="fp32"))
    assert lib.lbm_buffer_bytes(ctypes.byref(bad)) == 0
    h = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    assert b"4 GiB" in lib.lbm_last_error()
    # a narrow plane but a lattice row of the nine planes past 4 GiB (32-bit row offsets):
    # 119,304,704 FP32 columns (a multiple of 64) are the first whose row reaches 4 GiB
    for nx, ok_row in ((119_304_640, True), (119_304_704, False)):
        p = lbm.make_params(dict(nx=nx, ny=3, precision="fp32"))
        assert (lib.lbm_buffer_bytes(ctypes.byref(p)) != 0) == ok_row, nx
    assert lib.lbm_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert b"too wide" in lib.lbm_last_error()


def test_library_laplace_fit_matches_oracle(lib, oracle_mod):
    """lbm_laplace_fit (host FP64) against the oracle's fit on scattered drops, and its
    argument checks: no drop, a radius <= 0, a non-finite dp or radius."""
    import numpy as np

    rng = np.random.default_rng(9)
    R = rng.uniform(10.0, 80.0, 7)
    dp = 0.02 / R * (1 + 0.03 * rng.standard_normal(7))
    s, spread = lbm.laplace_fit(dp, R)
    s_o, spread_o = oracle_mod.laplace_fit(dp, R)
    assert abs(s / s_o - 1) < 1e-14 and abs(spread / spread_o - 1) < 1e-12
    for bad_dp, bad_r in (([], []), ([1e-3], [0.0]), ([1e-3], [-5.0]), ([float("nan")], [20.0]),
                          ([1e-3], [float("inf")])):
        with pytest.raises(lbm.LBMError):
            lbm.laplace_fit(bad_dp, bad_r)


def test_batch_arguments_are_rejected_before_device_use(lib):
    """An empty batch, a NULL parameter array, mixed EOS kinds or precisions and an
    invalid domain are refused on the host, before any device call."""
    good = lbm.make_params(dict(nx=16, ny=16, eos="cs", precision="fp32"))
    arr = (lbm.Params * 3)(good, good, good)
    h = ctypes.c_void_p()
    assert lib.lbm_batch_create(arr, 0, None, ctypes.byref(h)) == -1
    assert lib.lbm_batch_create(None, 3, None, ctypes.byref(h)) == -1
    for other in (dict(nx=16, ny=16, eos="vdw", K=0.3, T_over_Tc=0.9, precision="fp32"),
                  dict(nx=16, ny=16, eos="cs", precision="fp64"),
                  dict(nx=2, ny=16, eos="cs", precision="fp32")):
        arr[1] = lbm.make_params(other)
        assert lib.lbm_batch_create(arr, 3, None, ctypes.byref(h)) == -1
        assert not h.value
        assert b"batch" in lib.lbm_last_error()
