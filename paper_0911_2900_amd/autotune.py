"""Planning-tile autotuner.

The planning kernel's tile shape trades halo re-staging (small tiles stage
relatively more window cells) against parallelism (a scenario with few tiles
cannot fill 256 compute units) and lane utilisation (tiles with few agents
leave most of a 256-thread workgroup idle).  `tune` measures the planning
launch for each candidate shape on the caller's own scenarios, in the launch
form they will run in (one scenario alone, or all of them in one batched
launch), and returns the fastest.  `python -m paper_0911_2900_amd.autotune`
sweeps representative workloads and writes `tile_table.json`, which
`choose_tile` consults (nearest entry in v_m, log grid size and density) when
a caller leaves the tile open.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tile_table.json")

CANDIDATES = [(8, 8), (16, 8), (8, 16), (16, 16), (32, 8), (32, 16), (16, 32), (32, 32), (64, 8),
              (64, 16)]


def _time_plan(ctx, torch, hs, reps: int) -> float:
    """Median planning-kernel time (ms) over `reps` launches for handles hs,
    stamped by the launches themselves (the kernel's own start and end)."""
    torch.cuda.synchronize()
    ctx.timing_start(reps)
    for _ in range(reps):
        if len(hs) == 1:
            ctx.plan(hs[0])
        else:
            ctx.plan_batch(hs)
    ms = ctx.timing_read()
    return float(np.median(ms))


def tune(ctx, scenarios, candidates=None, reps: int = 31, warm_steps: int = 2):
    """Returns ((tx, ty), {tile: ms}) for the list of scenarios planned together."""
    import torch

    results = {}
    for tile in candidates or CANDIDATES:
        hs = [ctx.init_from(m, tile=tile) for m in scenarios]
        try:
            for _ in range(warm_steps):
                if len(hs) == 1:
                    ctx.plan(hs[0])
                    ctx.move(hs[0])
                else:
                    ctx.plan_batch(hs)
                    ctx.move_batch(hs)
            results[tile] = _time_plan(ctx, torch, hs, reps)
            # leave every scenario in a consistent state before destroying it
            if len(hs) == 1:
                ctx.move(hs[0])
            else:
                ctx.move_batch(hs)
        finally:
            for h in hs:
                ctx.destroy(h)
    best = min(results, key=results.get)
    return best, results


def _key(v: int, cells: int, density: float) -> dict:
    return {"v": int(v), "log2_cells": round(math.log2(max(cells, 1)), 2),
            "density": round(float(density), 3)}


# Scenarios with a speed per agent or several fields run the per-agent kernel
# (FP32 table path, a window per field).  On the 400 x 400 room with 40,000
# agents and speeds 1..5, launches took 9.6-10.2 us over tiles 16 x 8 .. 64 x 16;
# on the two-field counterflow hall 8.9-9.2 us; 32 x 8 is within 2 % of the
# best of both.
HET_TILE = (32, 8)


def choose_tile(v: int, width: int, height: int, n_agents: int, batched: bool = False,
                het: bool = False):
    """Tuned tile for a scenario (nearest table entry), or None without a table;
    het: the scenario has a speed per agent or several floor fields."""
    if het:
        return HET_TILE
    if not os.path.exists(TABLE):
        return None
    with open(TABLE) as f:
        table = json.load(f)["entries"]
    cells = width * height
    dens = n_agents / max(cells, 1)
    best, dist = None, None
    for e in table:
        if bool(e.get("batched", False)) != batched:
            continue
        d = (abs(e["v"] - v) * 4.0 + abs(e["log2_cells"] - math.log2(max(cells, 1)))
             + abs(e["density"] - dens) * 8.0)
        if dist is None or d < dist:
            best, dist = tuple(e["tile"]), d
    return best


def sweep(out_path: str = TABLE) -> dict:
    """Tune the representative workloads and write the table."""
    import torch

    from . import fast
    from . import scenarios as sc

    assert torch.cuda.is_available()
    ctx = fast.Context(device=0)
    entries = []

    def record(name, scen, batched):
        t0 = time.time()
        best, res = tune(ctx, scen)
        m = scen[0]
        e = dict(_key(m.v, m.W * m.H, m.n_agents / (m.W * m.H)), batched=batched, workload=name,
                 tile=list(best), ms={f"{a}x{b}": round(t, 5) for (a, b), t in res.items()})
        entries.append(e)
        print(f"{name}: best {best} {res[best]:.4f} ms ({time.time() - t0:.1f} s)", flush=True)

    for v in (1, 2, 3, 4, 5):
        record(f"room400_v{v}_40k", [sc.room(v=v)], False)
    record("room400_v4_10k", [sc.room(n_agents=10000, v=4)], False)
    record("room400_v4_80k", [sc.room(n_agents=80000, v=4)], False)
    for size, n in ((100, 2500), (200, 10000), (800, 160000)):
        record(f"room{size}_v4", [sc.room(n_agents=n, v=4, size=size)], False)
    record("large1000_v4_x4", [sc.large_member(k) for k in range(4)], True)
    record("room400_v4_x16", [sc.room(v=4, scn=k) for k in range(16)], True)
    record("ensemble_x64", [sc.ensemble_member(k) for k in range(64)], True)
    ctx.close()
    table = {"device": torch.cuda.get_device_name(0), "entries": entries}
    with open(out_path, "w") as f:
        json.dump(table, f, indent=1)
    return table


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else TABLE
    sweep(out)
