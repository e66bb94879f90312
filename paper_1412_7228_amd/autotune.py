"""Launch-shape autotuner for the step kernel and the batched engine.

Times candidate launch shapes on the GPU it runs on (HIP events on the
lattice's stream) and keeps the fastest.  Results are cached as JSON, keyed by
the device name and the workload's signature (lattice size, precision, EOS;
for a batch the sorted domain sizes), in ``$LBM_TUNE_CACHE`` or
``~/.cache/paper_1412_7228_amd/tune.json``.
"""
from __future__ import annotations

import hashlib
import json
import os

# (tile_x, tile_y, steps_per_pass)
LATTICE_CANDIDATES = [(256, 16, 1), (256, 64, 1), (128, 32, 1), (64, 32, 1),
                      (256, 8, 2), (256, 12, 2), (256, 16, 2), (256, 20, 2), (256, 24, 2), (256, 32, 2),
                      (128, 8, 2), (128, 16, 2), (128, 32, 2), (128, 64, 2)]
# (mode, tile_x, tile_y, steps_per_pass): per-step launches (one or two steps per
# launch) and the persistent launch (two steps per pass)
BATCH_CANDIDATES = [("per_step", 64, 16, 1), ("per_step", 64, 32, 1), ("per_step", 128, 16, 1),
                    ("per_step", 128, 8, 2), ("per_step", 128, 16, 2), ("per_step", 128, 32, 2),
                    ("per_step", 256, 8, 2), ("per_step", 256, 16, 2), ("per_step", 256, 32, 2),
                    ("persistent", 256, 16, 2), ("persistent", 256, 24, 2), ("persistent", 256, 32, 2)]


def cache_path() -> str:
    return os.environ.get("LBM_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1412_7228_amd", "tune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache: dict):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(p + ".tmp", p)
    except OSError:
        pass  # a read-only home only loses the cache


def _device() -> str:
    import torch

    return torch.cuda.get_device_name(0)


def _time(stream, fn, steps: int) -> float:
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def lattice_key(device: str, nx: int, ny: int, cfg: dict) -> str:
    return f"lattice|{device}|{nx}x{ny}|{cfg['precision']}|{cfg['eos']}"


def batch_key(device: str, shapes, cfg: dict) -> str:
    """Key of a batch: the device, the number of domains, a digest of the sorted domain
    sizes (a digest, not hash(): str hashes change from one Python process to the next),
    the precision and the EOS."""
    sizes = sorted(f"{ny}x{nx}" for ny, nx in shapes)
    sig = hashlib.sha1(",".join(sizes).encode()).hexdigest()[:12]
    return f"batch|{device}|{len(sizes)}|{sig}|{cfg['precision']}|{cfg['eos']}"


def tune_lattice(lat, steps: int = 40, candidates=None, use_cache: bool = True) -> dict:
    """Pick the fastest (tile_x, tile_y, steps_per_pass) for a Lattice (its state
    advances by the timing steps).  Returns {"tile": [tx, ty, spp], "ms": ...,
    "table": [...]} with ms per step."""
    key = lattice_key(_device(), lat.nx, lat.ny, lat.cfg)
    cache = _load() if use_cache else {}
    if key in cache and len(cache[key]["tile"]) == 3:
        lat.set_launch(*cache[key]["tile"])
        return cache[key]
    table = []
    for tx, ty, spp in candidates or LATTICE_CANDIDATES:
        if tx > 64 and lat.nx < tx - (6 if spp == 2 else 0):
            continue
        lat.set_launch(tx, min(ty, lat.ny), spp)
        lat.step(6)
        table.append(((tx, min(ty, lat.ny), spp), _time(lat.stream, lat.step, steps)))
    best = min(table, key=lambda t: t[1])
    lat.set_launch(*best[0])
    res = {"tile": list(best[0]), "ms": best[1], "table": [[list(t), m] for t, m in table]}
    cache[key] = res
    _store(cache)
    return res


def tune_batch(batch, steps: int = 20, candidates=None, use_cache: bool = True) -> dict:
    """Pick the fastest (mode, tile_x, tile_y, steps_per_pass) for a Batch (its
    state advances).  ms is per step."""
    key = batch_key(_device(), batch.shapes, batch.cfgs[0])
    cache = _load() if use_cache else {}
    if key in cache and len(cache[key]["launch"]) == 4:
        mode, tx, ty, spp = cache[key]["launch"]
        batch.set_launch(mode, tx, ty, steps_per_pass=spp)
        return cache[key]
    table = []
    for mode, tx, ty, spp in candidates or BATCH_CANDIDATES:
        batch.set_launch(mode, tx, ty, steps_per_pass=spp)
        batch.step(2)
        batch.sync()
        ms = _time(batch.stream, batch.step, steps)
        batch.sync()
        table.append(((mode, tx, ty, spp), ms))
    best = min(table, key=lambda t: t[1])
    mode, tx, ty, spp = best[0]
    batch.set_launch(mode, tx, ty, steps_per_pass=spp)
    res = {"launch": list(best[0]), "ms": best[1], "table": [[list(t), m] for t, m in table]}
    cache[key] = res
    _store(cache)
    return res
