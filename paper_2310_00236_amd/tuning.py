"""Tile-shape autotuner and its lookup table.

For a (physics, order, storage, compensation, size bucket) the tuner runs
every tile shape compiled into the library on the same problem, checks that
all of them give bit-identical fields (the kernels' results do not depend on
the tile shape), times them with HIP events, and records the fastest in
tune_table.json next to this file.  best_tile() reads that table; without an
entry it returns the first tile shape.
"""
from __future__ import annotations

import json
import os

import numpy as np

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")
ARCH = "gfx950"

_table = None


def size_bucket(nx: int, ny: int, nz: int = 1) -> str:
    cells = nx * ny * nz
    b = 1
    while b * 4 <= cells:
        b *= 4
    return f"{b}"


def key(physics, order, storage, comp, nx, ny, nz=1) -> str:
    return f"{ARCH}/{physics}/o{order}/{storage}/{comp}/{size_bucket(nx, ny, nz)}"


def _load():
    global _table
    if _table is None:
        _table = {}
        if os.path.exists(TABLE):
            with open(TABLE) as f:
                _table = json.load(f)
    return _table


def best_tile(physics, order, storage, comp, nx, ny, nz=1) -> int:
    t = _load()
    k = key(physics, order, storage, comp, nx, ny, nz)
    if k in t:
        return int(t[k]["tile"])
    # nearest size bucket with an entry for the same kernel kind
    prefix = k.rsplit("/", 1)[0] + "/"
    cand = [(abs(np.log(float(kk.rsplit("/", 1)[1]) / float(size_bucket(nx, ny, nz)))), v)
            for kk, v in t.items() if kk.startswith(prefix)]
    if cand:
        return int(min(cand, key=lambda c: c[0])[1]["tile"])
    return 0


def supported(problem, shape) -> bool:
    """Whether the library runs `problem` on kernel shape `shape` as given
    (8-bit compensation words do not run on the marching kind 1)."""
    return not (problem.comp == "twosum8" and problem.physics == "acoustic2d"
                and shape[3] == 1)


def tune(problem, material, fields, steps=50, reps=3, device="cuda:0",
         write=True):
    """Time every tile shape on `problem`; return (best_tile, timings_ms).

    Raises AssertionError if any two tile shapes give different bits."""
    import torch
    import paper_2310_00236_amd as hw
    tiles = hw.tiles(problem.physics)
    times, ref = {}, None
    for t in range(len(tiles)):
        if not supported(problem, tiles[t]):
            continue
        plan = hw.Plan(problem, device=device)
        plan.set_tile(t)
        plan.set_material(material)
        plan.set_fields(fields)
        plan.advance(2)                     # warm-up (code load, caches)
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.advance(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            best = ms if best is None else min(best, ms)
        times[t] = best
        out = plan.get_fields()
        plan.close()
        if ref is None:
            ref = out
        else:
            for k in ref:
                assert np.array_equal(ref[k], out[k]), \
                    f"tile {tiles[t]} changed the results of field {k}"
    best_t = min(times, key=times.get)
    if write:
        tab = dict(_load())
        k = key(problem.physics, problem.order, problem.storage, problem.comp,
                problem.nx, problem.ny, problem.nz)
        tab[k] = {"tile": best_t, "shape": list(tiles[best_t]),
                  "ms_per_step": {hw.tile_label(tiles[t]): v
                                  for t, v in times.items()}}
        with open(TABLE, "w") as f:
            json.dump(tab, f, indent=1, sort_keys=True)
        global _table
        _table = tab
    return best_t, times
