#!/usr/bin/env python3
"""Throughput of the fused pseudo-potential MRT lattice Boltzmann step on one MI355X.

Workload: a single 4096 x 4096 periodic lattice, spinodal decomposition from
the mean of the Carnahan-Starling coexistence densities at 0.7Tc
(rho = 0.183713 (1 + 0.01 xi), xi ~ U[-1, 1), seed 0), A = -0.5, kappa = 0,
FP32 distributions; the FP64 variant is measured beside it.  A lattice update
is the density/psi pass, force, pressure-tensor term, MRT collision and
streaming of one cell; the library's default launch fuses two time steps per
kernel launch (each launch reads and writes the state once).

Prints ONE JSON line:  value = MLUPS (million lattice updates per second).
roofline = the bound of the dominant kernel, HBM: with two steps per launch
the state is read once and written once per launch, so the algorithmic bytes
of a launch are 72 B (FP32) / 144 B (FP64) per cell; achieved = those bytes /
the measured launch time, against 8 TB/s; traffic = the HBM bytes per launch
that the FETCH_SIZE / WRITE_SIZE counters measured for this kernel in its
default shape (halo re-reads included), null in any other shape.  The fields
beside it give the same launch's vector-ALU view (FLOPS_PER_LU FP operations
per update against the 78.6 TFLOP/s vector peak without packed math) and the
bytes an unfused pair of single steps would have needed.  slab_share = the same
kernel on one GPU's share of the lattice cut into 8 y-slabs (4096 x 512 rows
plus 4 ghost rows per side), and the cost of refreshing the ghost rows.
cpu_baseline = the FP64 CPU oracle on every usable host core (count, quota and
model recorded) on a bounded sample of the same lattice, and on the 100^2 FP64
droplet end to end; it is the only leg that runs the oracle.  end_to_end = GPU
wall times from initial field to results (the same droplet between the
library's Maxwell densities; the 200^2 Laplace sweep; the benchmark lattice with
its host transfers).  copy_ceiling = a plain device copy (the library's
hand-written copy kernel and torch's), the practical HBM ceiling.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# vector ALU peak without packed math: 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz;
# the same for FP32 and FP64 on MI355X (the kernels are compiled without packed FP32)
ALU_PEAK_TFLOPS = {"fp32": 78.6, "fp64": 78.6}
FLOPS_PER_LU = 260  # FP arithmetic of one cell update in the single-step kernel's ISA
# HBM bytes per launch of the two-step kernel in the default shape on 4096^2,
# from rocprofv3 FETCH_SIZE + WRITE_SIZE (scaled by the copy calibration), and the
# VALU issue utilisation of the same launches (SQ_INSTS_VALU against 256 CUs x
# GRBM_GUI_ACTIVE / 8).  They hold for the kernel sources whose digest is
# COUNTERS_SOURCE_DIGEST; for any other build they are reported as null.
MEASURED_TRAFFIC = {("fp32", 256, 16): (763.2e6 + 617.5e6), ("fp64", 256, 69): (1347.1e6 + 1220.2e6)}
MEASURED_VALU_ISSUE = {("fp32", 256, 16): 0.831, ("fp64", 256, 69): 0.436}
COUNTERS_SOURCE_DIGEST = "d368bae567480736"
KERNEL_SOURCES = ("lbm_device.h", "lbm_internal.h", "lbm_tile.h", "lbm_tile2.h", "lbm_step.hip",
                  "../../include/lbm.h")  # the header fixes the state layout
from paper_1412_7228_amd import workloads  # noqa: E402  (data only: loads no library)

# the throughput lattice and the end-to-end droplet (paper_1412_7228_amd/workloads.json)
_LATTICE = workloads.get("lattice_4096_spinodal")
N = _LATTICE["lattice"][0]
RHO_MEAN = _LATTICE["rho_mean"]  # (rho_v + rho_l)/2 of CS at 0.7Tc
SPINODAL_NOISE, SPINODAL_SEED = _LATTICE["noise"], _LATTICE["seed"]
WORKLOAD = workloads.lattice_config("lattice_4096_spinodal")
_DROP = workloads.get("droplet_100")
DROPLET_100 = workloads.lattice_config("droplet_100")
DROP_R, DROP_W, DROP_NOISE, DROP_SEED = (_DROP["droplet"][k] for k in ("R", "W", "noise", "seed"))
DROP_STEPS = _DROP["steps"]
BYTES_PER_LU = {"fp32": 72, "fp64": 144}


def kernel_source_digest() -> str:
    """sha256 (first 16 hex digits) of the step kernel's sources and the header that
    fixes the state layout, in a fixed order."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1412_7228_amd", "csrc", name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def counters_current() -> bool:
    return kernel_source_digest() == COUNTERS_SOURCE_DIGEST


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--fp64-steps", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-slab", action="store_true", help="skip the one-GPU slab share measurement")
    ap.add_argument("--no-e2e", action="store_true", help="skip the end-to-end small workloads")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven droplet batch")
    ap.add_argument("--batch-steps", type=int, default=200, help="timed steps per batch launch mode")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--log", default=None, help="append the result as one JSON line to this file (default: $LBM_RUN_LOG, unset = no log)")
    ap.add_argument("--tile", type=str, default="", help="tile_x,tile_y of the step kernel")
    ap.add_argument("--copy-mib", type=int, default=2048,
                    help="size of the device-to-device copy timed as the practical bandwidth ceiling "
                         "(0 = skip); under a counter profiler it calibrates FETCH_SIZE/WRITE_SIZE")
    return ap.parse_args()


def copy_bandwidth(mib, reps=40):
    """The practical HBM ceiling: a device copy of `mib` MiB (read + write bytes / time),
    by the library's hand-written copy kernel (lbm_copy_bytes: one 16-byte load and store
    per lane) and by torch's copy, each timed with HIP events on torch's stream."""
    import ctypes

    import torch
    from paper_1412_7228_amd import lbm

    lib = lbm.load_library()
    n = mib * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def own():
        st = lib.lbm_copy_bytes(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                ctypes.c_size_t(n), stream)
        if st != 0:
            raise RuntimeError(f"lbm_copy_bytes failed: {st}")

    out = {}
    for name, fn in (("hand_written", own), ("torch", lambda: dst.copy_(src))):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = dict(ms=round(ms, 4), gbs=round(2 * n / (ms * 1e-3) / 1e9, 1))
    ok = bool(torch.equal(dst, src))
    del src, dst
    best = max(out.values(), key=lambda r: r["gbs"])["gbs"]
    return dict(bytes_per_copy=2 * n, gbs=best, kernels=out, copy_correct=ok)


def time_steps(lat, steps, warmup):
    """Launch `steps` steps on the lattice's stream bracketed by HIP events on that stream."""
    import torch

    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    s = lat.stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(s)
    lat.step(steps)
    t1.record(s)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)  # ms


def gpu_measure(precision, steps, warmup, tile):
    from paper_1412_7228_amd import inputs, lbm

    lat = lbm.Lattice(dict(WORKLOAD, precision=precision))
    if tile:
        lat.set_launch(*tile)
    lat.init_field(inputs.spinodal(N, N, RHO_MEAN, noise=SPINODAL_NOISE, seed=SPINODAL_SEED))
    spp = lat.launch[2]
    ms = time_steps(lat, steps, warmup)  # exactly `steps` (an odd count ends with one single step)
    ob = lat.observables(check=False)
    lus = float(N * N) * steps
    if steps % spp == 0:
        per_launch_s = ms * 1e-3 / (steps // spp)
    else:
        # the roofline is the fused kernel's: time whole launches of it on their own
        per_launch_s = time_steps(lat, max(spp, steps - steps % spp), 0) * 1e-3 / max(1, steps // spp)
    # bytes the launch must move: the state in and out once per launch
    gbs = BYTES_PER_LU[precision] * N * N / per_launch_s / 1e9
    tflops = FLOPS_PER_LU * N * N * spp / per_launch_s / 1e12
    tx, ty = lat.launch[0], lat.launch[1]
    fresh = counters_current()
    traffic = MEASURED_TRAFFIC.get((precision, tx, ty)) if (spp == 2 and fresh) else None
    roof = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=traffic,
                basis=f"launch minimum: the state read and written once per launch of {spp} steps, "
                      f"{BYTES_PER_LU[precision] // spp} B per update")
    roof["counters"] = dict(kernel_source_digest=kernel_source_digest(),
                            taken_on_digest=COUNTERS_SOURCE_DIGEST, current=fresh)
    # bytes per lattice update, counted explicitly: the method's 72 B (FP32) / 144 B (FP64)
    # per update, the fused launch's minimum (the state in and out once for spp updates)
    # and what the counters measured
    roof["bytes_per_update"] = dict(method=BYTES_PER_LU[precision],
                                    launch_minimum=round(BYTES_PER_LU[precision] / spp, 1),
                                    measured=round(traffic / (spp * N * N), 1) if traffic else None,
                                    updates_per_launch=spp * N * N)
    if traffic:
        roof["traffic_gbs"] = round(traffic / per_launch_s / 1e9, 1)
    if spp == 2:
        roof.update(unfused_equivalent_gbs=round(gbs * 2, 1),
                    frac_at_method_bytes=round(gbs * 2 / HBM_PEAK_GBS, 4),
                    frac_at_method_bytes_note=(
                        f"the method's {BYTES_PER_LU[precision]} B per update times the launch's "
                        f"{spp} x N^2 updates over the launch time; above 1 because one launch "
                        "advances two steps while reading and writing the state once (temporal "
                        "blocking), so the per-update byte count stops being a ceiling"),
                    alu=dict(achieved=round(tflops, 2), peak=ALU_PEAK_TFLOPS[precision], unit="TFLOP/s",
                             frac=round(tflops / ALU_PEAK_TFLOPS[precision], 4),
                             valu_issue_measured=MEASURED_VALU_ISSUE.get((precision, tx, ty)) if fresh else None))
    res = dict(ms_per_step=ms / steps, mlups=lus / (ms * 1e-3) / 1e6, steps=steps,
               launch_ms=per_launch_s * 1e3, roofline=roof, tile=list(lat.launch), mass=ob["mass"],
               n_nonfinite=ob["n_nonfinite"])
    lat.close()
    return res


def slab_share(launches=300, slabs=8, tiles=((0, 0), (256, 16), (256, 8), (128, 16), (128, 8))):
    """One GPU's share of the same lattice cut into `slabs` y-slabs: a 4096 x (4096/slabs)
    slab plus 4 ghost rows on each side, advanced with two steps per launch over its
    interior rows (lbm_step_rows), timed per launch shape with HIP events around each
    launch.  Between launches the ghost rows are refreshed as a neighbour would send them;
    here the slab is its own neighbour (periodic in y), which keeps it a valid lattice.
    exchange_bytes = what one launch needs from the two neighbours (9 planes x 4 rows each)."""
    import torch
    from paper_1412_7228_amd import inputs, lbm

    h, g = N // slabs, 4
    lat = lbm.Lattice(dict(WORKLOAD, ny=h + 2 * g, precision="fp32"))
    rho = inputs.spinodal(N, h, RHO_MEAN, noise=SPINODAL_NOISE, seed=SPINODAL_SEED)
    lat.init_field(np.concatenate([rho[-g:], rho, rho[:g]]))
    s = lat.stream
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def launch_and_refresh(timed):
        e = (ev(), ev()) if timed else None
        if e:
            e[0].record(s)
        lat.step_rows(2, g, h)
        if e:
            e[1].record(s)
        cur = lat.state_tensor()
        cur[:, :g] = cur[:, h:h + g]
        cur[:, h + g:] = cur[:, g:2 * g]
        return e

    for _ in range(200):  # clocks and caches settle before the first timed shape
        launch_and_refresh(False)
    shapes = []
    for tx, ty in tiles:
        lat.set_launch(tx, ty, 2)
        for _ in range(30):
            launch_and_refresh(False)
        evs = [launch_and_refresh(True) for _ in range(launches)]
        torch.cuda.synchronize()
        us = sum(a.elapsed_time(b) for a, b in evs) * 1e3 / launches
        shapes.append(dict(tile=list(lat.launch[:2]), launch_us=round(us, 2),
                           mlups=round(2 * N * h / us, 1)))
    best = min(shapes[1:], key=lambda r: r["launch_us"])
    # the same steps in three launches, as a slab that overlaps its ghost-row transfer
    # would run them: the rows that read no ghost row, then the two bands next to them
    lat.set_launch(*best["tile"], 2)
    inner, outer = [], []
    for k in range(30 + launches):
        e = [ev() for _ in range(4)]
        e[0].record(s)
        lat.step_rows(2, 2 * g, h - 2 * g, more=True)
        e[1].record(s)
        cur = lat.state_tensor()
        cur[:, :g] = cur[:, h:h + g]
        cur[:, h + g:] = cur[:, g:2 * g]
        e[2].record(s)
        lat.step_rows(2, g, g, more=True)
        lat.step_rows(2, h, g)
        e[3].record(s)
        if k >= 30:
            inner.append((e[0], e[1]))
            outer.append((e[2], e[3]))
    torch.cuda.synchronize()
    split = dict(interior_us=round(sum(a.elapsed_time(b) for a, b in inner) * 1e3 / launches, 2),
                 boundary_us=round(sum(a.elapsed_time(b) for a, b in outer) * 1e3 / launches, 2))
    ob = lat.observables(check=False)
    lat.close()
    return dict(slab=[N, h], ghost_rows=g, shapes=shapes, best=best, default=shapes[0], split=split,
                exchange_bytes=2 * 9 * g * N * 4, n_nonfinite=ob["n_nonfinite"])


def end_to_end():
    """Wall time of workloads from initial field to results on the GPU, with nothing from
    the oracle: the 100^2 FP64 droplet (CS, 0.8Tc, R = 25, 5000 steps) between the
    library's Maxwell densities (lbm_coexistence), the 200^2 Laplace sweep (R 20..60,
    T/Tc 0.6..0.8, kappa 0..0.6 at A = -0.5, plus the A = -0.9 rows at 0.6Tc; 60 drops,
    20,000 FP32 steps) as one batch, and the benchmark lattice including its host
    transfers (the rate with PCIe in it)."""
    import torch
    from paper_1412_7228_amd import inputs, laplace, lbm

    cfg = dict(DROPLET_100, precision="fp64")
    rv, rl = lbm.coexistence(cfg)
    rho = inputs.droplet(DROPLET_100["nx"], DROPLET_100["ny"], DROP_R, rl, rv, W=DROP_W, noise=DROP_NOISE, seed=DROP_SEED)
    torch.cuda.synchronize()
    t = time.perf_counter()
    lat = lbm.Lattice(cfg)
    lat.init_field(rho)
    lat.step(DROP_STEPS)
    ob_gpu = lat.observables()
    gpu_s = time.perf_counter() - t
    lat.close()
    # the benchmark lattice with its host transfers: initial density in (FP64, 134 MB),
    # 2000 steps, density field out (FP64)
    big = dict(WORKLOAD, precision="fp32")
    rho_big = inputs.spinodal(N, N, RHO_MEAN, noise=SPINODAL_NOISE, seed=SPINODAL_SEED)
    lat = lbm.Lattice(big)
    lat.init_field(rho_big)
    lat.step(20)
    lat.field("rho")  # first transfers warm the paths
    torch.cuda.synchronize()
    t = time.perf_counter()
    lat.init_field(rho_big)
    lat.step(2000)
    out = lat.field("rho")
    io_s = time.perf_counter() - t
    lat.close()
    cases = laplace.full_sweep_cases()
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = laplace.run_cases(cases, 20000, precision="fp32")
    sweep_s = time.perf_counter() - t
    return dict(droplet_100_fp64_5000=dict(gpu_s=round(gpu_s, 3), sigma_gpu=ob_gpu["sigma"],
                                           initial_densities="library (lbm_coexistence)"),
                laplace_sweep_200_fp32_20000=dict(drops=len(cases), gpu_s=round(sweep_s, 3),
                                                 two_phase=int(sum(r["ok"] for r in res))),
                lattice_4096_fp32_2000_with_host_io=dict(
                    s=round(io_s, 4), mlups=round(N * N * 2000 / io_s / 1e6, 1),
                    note="init_field from host FP64 + 2000 steps + density field back to host",
                    rho_finite=bool(np.isfinite(out).all())))


def uneven_batch(steps):
    """The uneven droplet batch (256 screened draws of the seeded stream, sides 64-512,
    about 25 M cells, FP32) in its two launch modes, timed with HIP events on the batch's
    stream after 10 untimed steps: per-step launches (256 x 16 tiles) and the persistent
    launch (its default 256 x 24 tiles).  Not the benchmark's value: the same kernel over
    uneven domains."""
    from paper_1412_7228_amd import batchbench, workloads

    w = workloads.get("uneven_batch_256")
    b, cases, cells, report = batchbench.build(w["domains"], w["seed"])
    modes = {}
    for mode, tile in (("per_step", (256, 16)), ("persistent", (256, 24))):
        ms = batchbench.time_mode(b, mode, tile, steps, steps_per_pass=2)
        modes[f"{mode}_{tile[0]}x{tile[1]}"] = dict(mlups=round(cells * steps / (ms * 1e-3) / 1e6, 1),
                                                    ms=round(ms, 3))
    obs = b.observables(check=False)
    b.close()
    return dict(domains=len(cases), cells=cells, timed_steps_per_mode=steps, modes=modes,
                redraws=report["redraws"] if report else None,
                domains_with_faults=sum(1 for o in obs if o["n_nonfinite"] > 0 or o["n_domain"] > 0))


def host_cores() -> dict:
    """The host's CPUs as this process sees them: nproc, the CPUs it may run on, the
    cgroup CPU quota, the CPU model; `usable` = the threads the oracle runs on."""
    info = dict(nproc=os.cpu_count() or 1)
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        info["affinity"] = info["nproc"]
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, period = fh.read().split()[:2]
            if q != "max":
                quota = float(q) / float(period)
    except (OSError, ValueError):
        pass
    info["cgroup_quota_cpus"] = quota
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    info["model"] = model
    usable = info["affinity"]
    if quota:
        usable = max(1, min(usable, int(quota)))
    info["usable"] = usable
    info["omp_num_threads_env"] = os.environ.get("OMP_NUM_THREADS")
    return info


def cpu_baseline(seconds):
    """The FP64 oracle (as it stands) on the host cores: (1) the full 4096^2 input, as many
    whole steps as fit in about `seconds`, on every usable core and on one thread; (2) the
    100^2 FP64 droplet of end_to_end (5000 steps, from the oracle's own Maxwell densities)
    end to end."""
    import oracle
    from paper_1412_7228_amd import inputs

    host = host_cores()
    nthr = host["usable"]
    o = oracle.Oracle(WORKLOAD, nthreads=nthr)
    o.init_field(inputs.spinodal(N, N, RHO_MEAN, noise=SPINODAL_NOISE, seed=SPINODAL_SEED))
    t = time.perf_counter()
    o.run(1)
    one = time.perf_counter() - t
    k = max(1, min(50, int(seconds / max(one, 1e-3)) - 1))
    t = time.perf_counter()
    o.run(k)
    dt = time.perf_counter() - t
    o.nthreads = 1
    t = time.perf_counter()
    o.run(1)
    one_thread = N * N / (time.perf_counter() - t) / 1e6
    del o
    e = oracle.thermo.carnahan_starling()
    _, Tc = oracle.thermo.critical_point(e)
    rv, rl = oracle.thermo.maxwell(e, DROPLET_100["T_over_Tc"] * Tc)
    rho = inputs.droplet(DROPLET_100["nx"], DROPLET_100["ny"], DROP_R, rl, rv, W=DROP_W, noise=DROP_NOISE, seed=DROP_SEED)
    t = time.perf_counter()
    d = oracle.Oracle(DROPLET_100, nthreads=nthr)
    d.init_field(rho)
    d.run(DROP_STEPS)
    ob = d.observables()
    e2e_s = time.perf_counter() - t
    return dict(value=N * N * k / dt / 1e6, unit="MLUPS", cores=nthr, kind="oracle",
                sample=f"4096x4096 lattice (the benchmark's input), {k} FP64 steps after 1 untimed, "
                       f"{dt:.1f} s on {nthr} threads",
                single_thread_mlups=round(one_thread, 2), host=host,
                droplet_100_fp64_5000=dict(oracle_s=round(e2e_s, 3), sigma_oracle=ob["sigma"],
                                           threads=nthr, initial_densities="oracle (thermo.maxwell)"))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported (the library has no "
              "multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    tile = tuple(int(v) for v in a.tile.split(",")) if a.tile else None  # tx,ty[,steps_per_pass]
    print(f"[bench] fp32 {N}x{N}: warmup {a.warmup}, timed {a.steps}", file=sys.stderr, flush=True)
    r32 = gpu_measure("fp32", a.steps, a.warmup, tile)
    print(f"[bench] fp32 {r32}", file=sys.stderr, flush=True)
    r64 = None
    if a.fp64_steps > 0:
        print(f"[bench] fp64 {N}x{N}: timed {a.fp64_steps}", file=sys.stderr, flush=True)
        r64 = gpu_measure("fp64", a.fp64_steps, a.warmup, tile)
        print(f"[bench] fp64 {r64}", file=sys.stderr, flush=True)
    slab = None
    if not a.no_slab:
        print("[bench] slab share (8 y-slabs)", file=sys.stderr, flush=True)
        slab = slab_share()
        print(f"[bench] slab {slab}", file=sys.stderr, flush=True)
    e2e = None
    if not a.no_e2e:
        print("[bench] end-to-end workloads", file=sys.stderr, flush=True)
        e2e = end_to_end()
        print(f"[bench] end-to-end {e2e}", file=sys.stderr, flush=True)
    batch = None
    if not a.no_batch:
        print("[bench] uneven droplet batch", file=sys.stderr, flush=True)
        batch = uneven_batch(a.batch_steps)
        print(f"[bench] batch {batch}", file=sys.stderr, flush=True)
    copy = None
    if a.copy_mib > 0:
        copy = copy_bandwidth(a.copy_mib)
        print(f"[bench] device copy {copy}", file=sys.stderr, flush=True)
    cpu = None
    if not a.no_cpu_baseline:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.cpu_seconds)
    line = {
        "metric": "MLUPS and % HBM roofline at 1 MI355X (FP32 vs FP64); runs to hit target sigma",
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": r32["steps"],
        "warmup": a.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "single 4096x4096 periodic lattice, spinodal decomposition, CS EOS, T/Tc=0.7, "
                        "A=-0.5, kappa=0, FP32 distributions",
            "lattice": [N, N],
            "launch": {"tile": r32["tile"][:2], "steps_per_pass": r32["tile"][2],
                       "launch_ms": r32["launch_ms"]},
        },
        "roofline": r32["roofline"],
        "fp64_variant": None if r64 is None else {
            "value": round(r64["mlups"], 1), "unit": "MLUPS", "steps": r64["steps"],
            "ms_per_step": r64["ms_per_step"], "launch": {"tile": r64["tile"][:2],
                                                          "steps_per_pass": r64["tile"][2]},
            "roofline": r64["roofline"],
        },
        "slab_share": slab,
        "end_to_end": e2e,
        "uneven_batch": batch,
        "cpu_baseline": cpu,
        "copy_ceiling": None if copy is None else {
            "gbs": copy["gbs"], "bytes": copy["bytes_per_copy"], "kernels": copy["kernels"],
            "copy_correct": copy["copy_correct"],
            "frac_of_peak": round(copy["gbs"] / HBM_PEAK_GBS, 4),
            "step_traffic_frac_of_copy": (round(r32["roofline"]["traffic_gbs"] / copy["gbs"], 4)
                                          if r32["roofline"].get("traffic_gbs") else None),
            "step_minimum_frac_of_copy": round(r32["roofline"]["achieved"] / copy["gbs"], 4),
            "note": "device-to-device copy, read + write bytes / time; the best of the library's "
                    "hand-written copy kernel and torch's copy"},
    }
    print(json.dumps(line), flush=True)
    from paper_1412_7228_amd import runlog

    runlog.append(dict(kind="bench", result=line), a.log)


if __name__ == "__main__":
    main()
