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
  wait, is at agent scope.
* The two-step kernels (lattice, per-step batch, persistent batch): a wave
  must pass every barrier its workgroup passes.  In the assembly every
  exec-masked region (the per-lane store guard) closes before any barrier or
  branch, so all barriers sit in scalar control flow; the persistent kernel's
  idle-wave path (waves of a narrow strip with no needed lane) is a loop of
  three barriers per row, as many as the busy waves pass."""
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


def _masked_regions(body):
    """Barriers reachable inside an exec-masked region: from each s_and_saveexec,
    every path of the control flow (fall-through and branches) is followed until
    the s_or_b64 exec restore of the same saved mask; a barrier met on the way
    would be skipped by a wave whose mask is empty."""
    lines = [l.strip() for l in body]
    labels = {l.split(":")[0]: k for k, l in enumerate(lines) if l.startswith(".LBB")}
    bad = []
    for k, l in enumerate(lines):
        m = re.match(r"s_and_saveexec_b64\s+(s\[\d+:\d+\])", l)
        if not m:
            continue
        restore = "s_or_b64 exec, exec, " + m.group(1)
        todo, seen = [k + 1], set()
        while todo:
            q = todo.pop()
            while q < len(lines) and q not in seen:
                seen.add(q)
                t = lines[q]
                if t.startswith(restore) or t.startswith("s_endpgm"):
                    break
                if t.startswith("s_barrier"):
                    bad.append((k, q))
                    break
                if t.startswith("s_branch"):
                    q = labels[t.split()[1]]
                    continue
                if t.startswith("s_cbranch"):
                    todo.append(labels[t.split()[1]])
                q += 1
    return bad


@pytest.mark.parametrize("src,prefix,count", [
    ("lbm_step.hip", "_ZN3lbm7k_step2I", 32),
    ("lbm_batch.hip", "_ZN3lbm13k_batch_step2I", 16),
    ("lbm_persistent.hip", "_ZN3lbm18k_batch_persistentI", 16),
])
def test_two_step_kernels_reach_every_barrier_in_scalar_control_flow(tmp_path, src, prefix, count):
    fns = _functions(_assembly(os.path.join(CSRC, src), tmp_path), prefix)
    assert len(fns) == count
    for name, body in fns.items():
        assert sum("s_barrier" in l for l in body) >= 12, name  # 3 per row, 2 rows unrolled, 2 directions
        assert _masked_regions(body) == [], name


def test_persistent_idle_waves_pass_three_barriers_per_row(tmp_path):
    fns = _functions(_assembly(os.path.join(CSRC, "lbm_persistent.hip"), tmp_path), "_ZN3lbm18k_batch_persistentI")
    for name, body in fns.items():
        ops = [l.split()[0] for l in (x.strip() for x in body) if l and not l.startswith((";", "."))]
        triples = sum(1 for k in range(len(ops) - 2) if ops[k:k + 3] == ["s_barrier"] * 3)
        assert triples >= 1, name


def test_barrier_check_finds_a_barrier_in_a_divergent_branch(tmp_path):
    fns = _functions(_assembly(os.path.join(PROTO, "barrier_in_branch.hip"), tmp_path), "_Z19k_barrier_in_branch")
    assert len(fns) == 1
    body = next(iter(fns.values()))
    assert any("s_barrier" in l for l in body)
    assert _masked_regions(body) != []
