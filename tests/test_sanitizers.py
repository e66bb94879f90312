"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle is rebuilt with gcc's sanitizers into a temporary directory and
driven from a child Python process with the sanitizer runtimes preloaded; any
out-of-bounds access, use after free, signed overflow or misaligned access
aborts the child.  Its results must equal those of the normal build.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import json, sys
sys.path.insert(0, sys.argv[2])
import numpy as np
import oracle
if sys.argv[1] != "-":
    oracle._LIB = oracle._SRC = sys.argv[1]  # the sanitized build; never rebuilt here
from paper_1412_7228_amd import inputs
out = {}
for eos, T in (("cs", 0.8), ("vdw", 0.9), ("pr", 0.8), ("ideal", 0.8)):
    cfg = dict(nx=23, ny=17, eos=eos, T_over_Tc=T, A=-0.4, kappa=0.3)
    o = oracle.Oracle(cfg, nthreads=2)
    o.init_field(inputs.spinodal(23, 17, 0.2, noise=1e-2, seed=3),
                 0.01 * np.ones((17, 23)), -0.02 * np.ones((17, 23)))
    o.run(4)
    f = o.f_soa()
    o.set_f_soa(f)
    o.run(1)
    fl = o.fields()
    ob = o.observables()
    it = o.interaction(fl["rho"])
    c = o.collide_cell(np.linspace(0.01, 0.09, 9), F=(1e-3, -2e-3), Q=(1e-4, 2e-4, -3e-4))
    out[eos] = dict(mass=ob["mass"], f=o.f_soa().ravel()[::7].tolist(),
                    Fx=np.asarray(it["Fx"]).ravel()[::5].tolist(), cell=np.asarray(c).tolist())
print(json.dumps(out))
"""


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-D_DEFAULT_SOURCE", "-o", str(lib), os.path.join(ROOT, "oracle", "lbm_oracle.c"),
                           "-lm"])
    drv = tmp_path / "driver.py"
    drv.write_text(DRIVER)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    san = subprocess.run([sys.executable, str(drv), str(lib), ROOT], capture_output=True, text=True,
                         env=env, timeout=600)
    assert san.returncode == 0, san.stderr[-4000:]
    plain = subprocess.run([sys.executable, str(drv), "-", ROOT], capture_output=True, text=True,
                           timeout=600)
    assert plain.returncode == 0, plain.stderr[-4000:]
    a, b = json.loads(san.stdout), json.loads(plain.stdout)
    for eos in a:
        for k in a[eos]:
            x, y = np.asarray(a[eos][k]), np.asarray(b[eos][k])
            assert np.allclose(x, y, rtol=1e-12, atol=1e-15), (eos, k)
