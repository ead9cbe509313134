"""Launch-shape tuner of the merged step (qed_plan_*).

The merged step has four runtime launch parameters (``qed_plan_config``): particles per
streaming block, streaming blocks per processing block, the cap on the blocks of one set, and
the photon pass's compiled variant (tile size and waves per SIMD; single precision).
Which values are fastest depends on the workload (set sizes, the share of transitions, how
the photon population grows over a run) and on the device, so they are chosen by timing the
caller's own workload.  A search is coordinate-wise: each parameter in turn is swept with the
others held at the best values so far, and a value replaces the one held only when it is
faster by more than a margin (1%: closer timings are within the run-to-run noise, and a
search that followed them would pick a different shape on each run).  Results are cached per (workload key, device name,
library build) in memory and, when a path is given, in a JSON file, so a second tuning of the
same workload on the same device and build costs nothing.

Used by ``sim.Simulation.tune`` / ``sim.Batch.tune`` and by the benchmark.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

# the plan's runtime launch parameters and the values swept (0 = the library's default:
# one resident round of blocks per set)
SPACE = {
    "particles_per_block": (256, 512, 1024, 2048),
    "process_group": (2, 4, 8),
    "max_blocks_per_set": (0, 2048),
    "photon_variant": (0, 1, 2),   # photon pass: 1024-slot tiles, 512-slot tiles, 1024 prefetching at 3 waves/SIMD
}
DEFAULT = {"particles_per_block": 1024, "process_group": 4, "max_blocks_per_set": 0, "photon_variant": 0}

_memory: dict = {}


def device_key():
    """Device name and the build of the library (its file's size and modification time)."""
    import torch

    from . import LIB_PATH
    st = os.stat(LIB_PATH)
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{name}|{st.st_size}|{int(st.st_mtime)}"


def cache_key(workload_key: str, dev: str | None = None) -> str:
    return hashlib.sha256(f"{workload_key}||{dev if dev is not None else device_key()}".encode()).hexdigest()[:24]


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(workload_key: str, run, space=None, start=None, cache_path=None, order=None, log=None, margin=0.01):
    """Coordinate search over ``space`` (dict name -> candidate values).  ``run(cfg)`` executes the
    workload with launch configuration ``cfg`` (a dict with every name of the space) and returns
    its wall time in seconds; a value replaces the one held when its time is below
    (1 - ``margin``) times the held one's.  Returns (best cfg, {"cfg as text": seconds} of every
    timing made, cached flag)."""
    space = dict(SPACE if space is None else space)
    key = cache_key(workload_key)
    if key in _memory:
        return dict(_memory[key]["best"]), dict(_memory[key]["timings"]), True
    if cache_path:
        hit = _read(cache_path).get(key)
        if hit:
            _memory[key] = hit
            return dict(hit["best"]), dict(hit["timings"]), True
    best = {k: (start or DEFAULT).get(k, v[0]) for k, v in space.items()}
    timings = {}

    def measure(cfg):
        label = json.dumps(cfg, sort_keys=True)
        if label not in timings:
            t0 = time.perf_counter()
            wall = run(dict(cfg))
            timings[label] = float(wall)
            if log:
                log(f"autotune {workload_key}: {label} -> {wall:.4f} s ({time.perf_counter() - t0:.2f} s incl. setup)")
        return timings[label]

    for name in (order or list(space)):
        held = measure(best)
        vals = {}
        for v in space[name]:
            cfg = dict(best)
            cfg[name] = v
            vals[v] = measure(cfg)
        cand = min(vals, key=vals.get)
        if vals[cand] < (1.0 - margin) * held:
            best[name] = cand
    entry = {"workload": workload_key, "best": best, "timings": timings}
    _memory[key] = entry
    if cache_path:
        data = _read(cache_path)
        data[key] = entry
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, cache_path)
    return dict(best), timings, False
