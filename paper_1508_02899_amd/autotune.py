"""Autotuner for the batched 1D form.

For every velocity-capacity class present in a batch (members with
nv <= 9, 17, 33, 65, 129), time candidate work decompositions -- lanes per
tile (64, 128, 256: one lane per site), or split-column tiles (block 0:
each column over several lanes, for classes whose members all have
nv == cap), and resident workgroups per compute unit of the persistent
launch (0 = one workgroup per tile) -- on the GPU with HIP events, on a
sub-batch holding only that class's members, and keep the fastest.  Then,
for batches that allow it, time the whole batch under the per-step
schedule and under the resident one (a single launch per call with
per-member step barriers) and keep the faster.  Results are cached as JSON keyed by GPU architecture, class,
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
    sched = tune_schedule(batch, flows, scheme, steps, graph_steps, cache,
                          use_cache, log)
    if sched is not None:
        chosen["schedule"] = sched
        dirty = dirty or sched[3]
    if dirty and use_cache:
        save_cache(cache, cache_path)
    return chosen


RESIDENT_CAPS = (17, 33, 65, 129)
# (workgroups per CU (0: as many as fit), items per work-counter fetch)
RESIDENT_CANDIDATES = ((0, 4), (0, 8), (0, 16), (0, 32), (0, 64), (2, 16))
# the schedules are compared over this many steps, the per-step one
# replaying a graph of as many (as a long run does)
SCHEDULE_STEPS = 50


def tune_schedule(batch, flows, scheme, steps, graph_steps, cache, use_cache,
                  log=None):
    """With the per-class decompositions applied, time the whole batch
    under the per-step schedule (graph replays) and the resident schedule
    (each grid of RESIDENT_GRIDS) and keep the faster; only for batches
    whose members all have nv in RESIDENT_CAPS (else None).  Returns
    (mode name, grid_per_cu, ms_per_step, newly timed)."""
    import numpy as np
    import torch

    from .lattice import PER_STEP, RESIDENT
    if not all(m.nv in RESIDENT_CAPS for m in batch.members):
        return None
    key = (f"{_arch()}|schedule|{scheme}|n{len(batch.members)}|"
           f"2^{int(round(math.log2(max(batch.total_cells, 1))))}")
    if use_cache and key in cache:
        c = cache[key]
        if c["mode"] == "resident":
            batch.schedule(RESIDENT, c["grid_per_cu"], c.get("chunk", 0))
        else:
            batch.schedule(PER_STEP)
        return (c["mode"], c["grid_per_cu"], c.get("ms_per_step"), False)
    rng = np.random.default_rng(0)
    f = torch.from_numpy(batch.pack_state(
        [rng.random((m.nv, m.nx)).astype(np.float32)
         for m in batch.members])).cuda()
    u = torch.from_numpy(batch.pack_flow(flows)).cuda()
    n = min(SCHEDULE_STEPS,
            min(max(1, (m.n_u_slices * m.u_hold) if m.u_hold else
                    SCHEDULE_STEPS) for m in batch.members))
    n = max(2, n - n % 2)
    g = n

    def timed():
        batch.step(f, u, 2)  # warm-up (captures nothing: 2 eager steps)
        batch.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        batch.step(f, u, n, graph_steps=g)
        e1.record()
        torch.cuda.synchronize()
        batch.sync()
        return e0.elapsed_time(e1) / n

    batch.schedule(PER_STEP)
    best = ("per_step", g, timed())
    if log:
        log(f"autotune schedule: per step (graph of {g}): {best[2]:.4f} ms")
    chunk = 0
    for gpc, ck in RESIDENT_CANDIDATES:
        try:
            batch.schedule(RESIDENT, gpc, ck)
        except Exception as e:  # noqa: BLE001 - a schedule that does not fit
            if log:
                log(f"autotune schedule: resident {gpc}/CU refused: {e}")
            continue
        ms = timed()
        if log:
            log(f"autotune schedule: resident, {gpc} workgroups per CU "
                f"(0 = as many as fit), chunks of {ck}: {ms:.4f} ms")
        if ms < best[2]:
            best, chunk = ("resident", gpc, ms), ck
    if best[0] == "resident":
        batch.schedule(RESIDENT, best[1], chunk)
    else:
        batch.schedule(PER_STEP)
    del f, u
    cache[key] = {"mode": best[0], "grid_per_cu": best[1], "chunk": chunk,
                  "ms_per_step": round(best[2], 5)}
    return (best[0], best[1], best[2], True)
