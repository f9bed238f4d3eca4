"""Autotuner of the batch schedule and tile.

A batch of trajectories can run in the spread schedule (each trajectory over
ceil(d_r / k) workgroups of k resonator layers: the tile height k) or in the
packed schedule (one workgroup per FP64 trajectory).  Which is faster depends
on the shapes and on how many trajectories there are, so the tuner measures:
for each candidate it runs a short prefix of the batch (a few RK4 steps of
every trajectory, from copies of the inputs, after one untimed run of the same
configuration) and keeps the fastest in RK steps x trajectories / s.  Results
are cached per batch signature (the multiset of shapes, precisions and the
trajectory count) in memory and, if a path is given, in a JSON file.

Candidates: spread with tile heights 1, 2, 3, 4 (the library lowers a height
that does not fit the kernel's register rows or LDS; a height above every
trajectory's d_r repeats a smaller one and is skipped) and packed.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional

from . import lr

_MEM: Dict[str, dict] = {}


def signature(items) -> str:
    """Batch signature: sorted shapes (d_q, d_r, d_f, M, precision) with counts."""
    counts: Dict[tuple, int] = {}
    for it in items:
        m = it["model"]
        k = (m.d_q, m.d_r, m.d_f, int(it["M"]), int(it.get("precision", 0)))
        counts[k] = counts.get(k, 0) + 1
    return ";".join(f"{k[0]}x{k[1]}x{k[2]}:M{k[3]}:p{k[4]}*{c}" for k, c in sorted(counts.items()))


def candidates(max_layers: int = 4) -> List[dict]:
    out = [{"schedule": "spread", "layers": k} for k in range(1, max_layers + 1)]
    out.append({"schedule": "packed", "layers": 0})
    return out


def flags_of(cand: dict) -> int:
    if cand["schedule"] == "packed":
        return lr.LR_BATCH_PACKED
    return lr.LR_BATCH_SPREAD_LAYERS(cand["layers"])


def _measure(items, cand, steps, stream):
    import torch
    trial = []
    for it in items:
        t = dict(it)
        t["nsteps"] = min(int(it["nsteps"]), steps)
        t["B"] = it["B"].clone()
        t["obs_stride"] = 0
        t.pop("obs", None)
        trial.append(t)
    b = lr.Batch(trial, stream=stream, flags=flags_of(cand))
    b.run()  # untimed: first launch of this configuration
    if b.status()[0] != lr.LR_OK:
        b.close()
        return None
    for t, it in zip(trial, items):
        t["B"].copy_(it["B"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    rc = b.status()[0]
    el = time.perf_counter() - t0
    b.close()
    if rc != lr.LR_OK:
        return None
    return sum(t["nsteps"] for t in trial) / el


def tune(items, steps: int = 20, stream=None, cache_path: Optional[str] = None, max_layers: int = 4) -> dict:
    """Pick the schedule and tile for `items` (lr.Batch item dicts; their device
    tensors are only read).  Returns {"schedule", "layers", "flags", "rates"}."""
    sig = signature(items)
    disk = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            disk = json.load(fh)
    if sig in _MEM:
        return _MEM[sig]
    if sig in disk:
        _MEM[sig] = disk[sig]
        return disk[sig]
    rates = {}
    seen_tiles = set()
    for cand in candidates(max_layers):
        if cand["schedule"] == "spread":
            # effective tile per trajectory after the library's lowering
            eff = tuple(min(cand["layers"], it["model"].d_r) for it in items)
            if eff in seen_tiles:
                continue
            seen_tiles.add(eff)
        key = f'{cand["schedule"]}:{cand["layers"]}'
        try:
            rates[key] = _measure(items, cand, steps, stream)
        except lr.LrError:
            rates[key] = None
    ok = {k: v for k, v in rates.items() if v is not None}
    if not ok:
        raise RuntimeError("no candidate configuration runs this batch")
    best = max(ok, key=ok.get)
    sched, layers = best.split(":")
    res = {"schedule": sched, "layers": int(layers), "flags": flags_of({"schedule": sched, "layers": int(layers)}),
           "rates": rates, "steps": steps}
    _MEM[sig] = res
    if cache_path:
        disk[sig] = res
        with open(cache_path, "w") as fh:
            json.dump(disk, fh, indent=1)
    return res


def tuned_batch(items, stream=None, steps: int = 20, cache_path: Optional[str] = None) -> "lr.Batch":
    """lr.Batch of `items` in the configuration the tuner picks."""
    res = tune(items, steps=steps, stream=stream, cache_path=cache_path)
    return lr.Batch(items, stream=stream, flags=res["flags"])
