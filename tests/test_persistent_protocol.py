"""CPU checks of the batched engine's persistent launch (the kernel in
paper_1412_7228_amd/csrc/lbm_persistent.hip), before and besides its GPU tests.

* The scheduling protocol (per-XCD queues handing out tiles pair by pair, a
  per-domain counter as the step barrier, bounded waits that abort through an
  error flag) modelled with host threads as workgroups, under random delays at
  every step: every run ends, every domain is exactly between two pairs
  whenever one of its tiles starts, and a stalled producer ends the launch
  through the error flag instead of hanging it.  A model with a barrier target
  one pair short is caught by the same checks.
* The compiled kernel: an earlier form of the barrier wait, a loop run by
  thread 0 alone inside a thread-0 section, never finished on the GPU.  A loop
  whose continuation depends on which lanes of a wave are active shows in
  gfx950 assembly as an exec mask narrowed inside the loop
  (s_andn2_b64 exec, exec, ...).  The fixture with that wait shape shows it;
  the library's persistent kernel, whose every loop test is on scalar values,
  must not, in any instantiation; and its one cache invalidation, after a
  wait, is at agent scope."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROTO = os.path.join(HERE, "protocol")
CSRC = os.path.join(ROOT, "paper_1412_7228_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


def _model(tmp_path, src):
    exe = str(tmp_path / "model")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe, src])
    return exe


def test_protocol_model_ends_and_keeps_every_domain_between_two_pairs(tmp_path):
    exe = _model(tmp_path, os.path.join(PROTO, "persistent_protocol.cpp"))
    res = subprocess.run([exe, "1", "30"], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "0 failures" in res.stdout


def test_protocol_model_catches_a_barrier_one_pair_short(tmp_path):
    src = open(os.path.join(PROTO, "persistent_protocol.cpp")).read()
    bad = src.replace("const unsigned target = (unsigned)b.ntiles[d] * s;",
                      "const unsigned target = (unsigned)b.ntiles[d] * (s - 1);")
    assert bad != src
    path = tmp_path / "bad.cpp"
    path.write_text(bad)
    exe = _model(tmp_path, str(path))
    res = subprocess.run([exe, "1", "10"], capture_output=True, text=True, timeout=120)
    assert res.returncode == 1 and "barrier violations" in res.stdout


def _assembly(src, tmp_path):
    if HIPCC is None:
        pytest.skip("hipcc not found")
    out = str(tmp_path / (os.path.basename(src) + ".s"))
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=on",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           "--cuda-device-only", "-S", src, "-o", out],
                          stderr=subprocess.DEVNULL)
    return open(out).read().splitlines()


def _functions(lines, prefix):
    """{symbol: body lines} of the functions whose symbol starts with prefix."""
    out = {}
    for i, l in enumerate(lines):
        m = re.match(r"^(" + re.escape(prefix) + r"\w*):", l)
        if m:
            j = i
            while not lines[j].startswith(".Lfunc_end"):
                j += 1
            out[m.group(1)] = lines[i:j]
    return out


NARROWED = re.compile(r"s_andn2_b64\s+exec,\s*exec")


def test_thread0_wait_loop_fixture_shows_a_lane_dependent_loop(tmp_path):
    fns = _functions(_assembly(os.path.join(PROTO, "thread0_wait_loop.hip"), tmp_path), "_Z14k_thread0_wait")
    assert len(fns) == 1
    body = next(iter(fns.values()))
    assert any(NARROWED.search(l) for l in body)
    assert any("s_sleep" in l for l in body)


def test_persistent_kernel_has_no_lane_dependent_loop(tmp_path):
    fns = _functions(_assembly(os.path.join(CSRC, "lbm_persistent.hip"), tmp_path), "_ZN3lbm18k_batch_persistent")
    assert len(fns) == 16  # FP32/FP64 x 4 EOS x 128/256 lanes
    for name, body in fns.items():
        assert not any(NARROWED.search(l) for l in body), name
        assert any("s_sleep" in l for l in body), name  # the wait loop is there
        assert sum("s_barrier" in l for l in body) >= 4, name
        # the consumer's L1 is invalidated at agent scope (the workgroup-scope form,
        # buffer_inv sc0, leaves the L1 as it is outside thread-group-split mode)
        invs = [l.split()[1:] for l in body if l.strip().startswith("buffer_inv")]
        assert invs == [["sc1"]], (name, invs)
