"""Autotuner for the batched 1D form.

For every velocity-capacity class present in a batch (members with
nv <= 9, 17, 33, 65, 129), time candidate work decompositions -- lanes per
tile (64, 128, 256: one lane per site), or split-column tiles (block 0:
each column over several lanes, for classes whose members all have
nv == cap), and resident workgroups per compute unit of the persistent
launch (0 = one workgroup per tile) -- on the GPU with HIP events, on a
sub-batch holding only that class's members, and keep the fastest.  Results are cached as JSON keyed by GPU architecture, class,
scheme and the class's size (log2 of its cell count), so later batches of
similar shape reuse them without timing.
"""
from __future__ import annotations

import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning", "batch1d.json")

CANDIDATES = [(64, 0), (128, 0), (256, 0), (64, 2), (64, 4), (64, 8),
              (128, 1), (128, 2), (128, 4), (256, 1), (256, 2)]
# split-column tiles (block 0), for the classes that allow them
SPLIT_CANDIDATES = [(0, 0), (0, 2), (0, 4), (0, 8)]
SPLIT_CAPS = (17, 33, 65, 129)
DEFAULT = (256, 0)


def candidates(cap: int, nvs) -> list:
    """Decompositions to time for a class with capacity cap whose members
    have the velocity counts nvs."""
    if cap in SPLIT_CAPS and all(nv == cap for nv in nvs):
        return CANDIDATES + SPLIT_CANDIDATES
    return list(CANDIDATES)


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _key(arch: str, cap: int, scheme: str, cells: int) -> str:
    return f"{arch}|cap{cap}|{scheme}|2^{int(round(math.log2(max(cells, 1))))}"


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def save_cache(cache: dict, path: str = CACHE) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def classes_of(members):
    from .lattice import Batch
    out = {}
    for i, m in enumerate(members):
        cap = next(c for c in Batch.CAPS if m.nv <= c)
        out.setdefault(cap, []).append(i)
    return out


def _time_class(sub, f, u, steps, graph_steps, block, gpc):
    import torch
    sub.tune(sub_cap(sub), block, gpc)
    sub.step(f, u, 2)  # warm-up
    sub.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sub.step(f, u, steps, graph_steps=graph_steps)
    e1.record()
    torch.cuda.synchronize()
    sub.sync()
    return e0.elapsed_time(e1) / steps


def sub_cap(sub):
    from .lattice import Batch
    return next(c for c in Batch.CAPS if max(m.nv for m in sub.members) <= c)


def tune_batch(batch, flows, scheme: str = "koren", steps: int = 20,
               graph_steps: int = 10, use_cache: bool = True,
               cache_path: str = CACHE, log=None) -> dict:
    """Pick (block, grid_per_cu) per class for ``batch`` and apply it.

    ``flows``: per-member flow arrays (numpy, [slices, nx]) used for the
    timing runs.  Returns {cap: (block, grid_per_cu, ms_per_step or None)}.
    """
    import numpy as np
    import torch

    from .lattice import Batch
    arch = _arch()
    cache = load_cache(cache_path) if use_cache else {}
    chosen = {}
    dirty = False
    for cap, idx in sorted(classes_of(batch.members).items()):
        cells = sum(batch.members[i].nx * batch.members[i].nv for i in idx)
        nvs = [batch.members[i].nv for i in idx]
        # classes that admit split-column tiles have more candidates
        key = _key(arch, cap, scheme, cells) + (
            "|split" if len(candidates(cap, nvs)) > len(CANDIDATES) else "")
        if use_cache and key in cache:
            blk, gpc = cache[key]["block"], cache[key]["grid_per_cu"]
            chosen[cap] = (blk, gpc, cache[key].get("ms_per_step"))
            batch.tune(cap, blk, gpc)
            continue
        mems = [batch.members[i] for i in idx]
        sub = Batch(mems, scheme=scheme, stream=batch.stream)
        rng = np.random.default_rng(0)
        f = torch.from_numpy(sub.pack_state(
            [rng.random((m.nv, m.nx)).astype(np.float32) for m in mems])).cuda()
        u = torch.from_numpy(sub.pack_flow([flows[i] for i in idx])).cuda()
        n = min(steps, min(max(1, (m.n_u_slices * m.u_hold) if m.u_hold else
                              steps) for m in mems))
        n -= n % 2
        best = None
        for blk, gpc in candidates(cap, [m.nv for m in mems]):
            ms = _time_class(sub, f, u, max(n, 2), min(graph_steps, max(n, 2)),
                             blk, gpc)
            if log:
                log(f"autotune cap {cap}: block {blk} gpc {gpc}: {ms:.4f} ms")
            if best is None or ms < best[2]:
                best = (blk, gpc, ms)
        sub.close()
        chosen[cap] = best
        batch.tune(cap, best[0], best[1])
        cache[key] = {"block": best[0], "grid_per_cu": best[1],
                      "ms_per_step": round(best[2], 5)}
        dirty = True
    if dirty and use_cache:
        save_cache(cache, cache_path)
    return chosen
