"""Seeded synthetic scenario generators (inputs only).

These build the cell-type grids (0 free, 1 wall, 2 exit; row-major, shape
(H, W)) and the run parameters of the workloads that stand in for the paper's
unstated geometry: the paper times 396 one-second steps with k_S = 1.2,
k_other = 0, one v_m for all agents and focuses on v_m = 4 and 40,000 agents
(Sec. 2 and Sec. 3).  Cells are 0.4 m.  Randomness comes from numpy's PCG64
streams seeded per scenario, so this module holds none of the model's own
arithmetic (no floor field, no weights, no Philox): it serves the product path
and the test oracle alike, and both receive the very same grids.

Workloads:
  corridor      60 x 25 cells, border walls, a 3-cell exit in the right wall
                (x = 59, y = 11..13); 200 agents, v_m = 4, seed 1.
  room          400 x 400 cells, border walls, a 10-cell exit in the right
                wall (x = 399, y = 195..204); 40,000 agents; v_m = 1..5.
  ensemble      256 scenarios: W, H ~ U{30..300}; 0-15 % random rectangular
                pillars (sides 1..4) kept 2 cells away from exits; 1-4 exits of
                width 2..10 on random sides; N log-uniform in [50, 20000],
                clamped to half the free cells; v_m ~ U{1..5}.
  large         16 scenarios of 1000 x 1000 cells with 10 % pillars and four
                10-cell exits centred on each side; 200,000 agents, v_m = 4.
  fd_corridor   fundamental-diagram corridor: 100 x 10 free cells (40 m x 4 m)
                in border walls, the whole right wall an exit, agents on
                uniformly drawn cells of the first 50 columns at a given
                density; a 10-column measurement area (x = 61..70) and the
                region upstream of the line between columns 70 and 71.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FREE, WALL, EXIT = 0, 1, 2


@dataclass
class Scenario:
    name: str
    cell_type: np.ndarray          # uint8 (H, W)
    n_agents: int
    v: int
    k_s: float = 1.2
    seed: int = 1
    scn: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def W(self) -> int:
        return int(self.cell_type.shape[1])

    @property
    def H(self) -> int:
        return int(self.cell_type.shape[0])


def walled_box(W: int, H: int) -> np.ndarray:
    t = np.zeros((H, W), dtype=np.uint8)
    t[0, :] = WALL
    t[-1, :] = WALL
    t[:, 0] = WALL
    t[:, -1] = WALL
    return t


def corridor(n_agents: int = 200, v: int = 4, seed: int = 1, scn: int = 0) -> Scenario:
    t = walled_box(60, 25)
    t[11:14, 59] = EXIT
    return Scenario("corridor_60x25", t, n_agents, v, 1.2, seed, scn)


def room(n_agents: int = 40000, v: int = 4, seed: int = 1, scn: int = 0,
         size: int = 400) -> Scenario:
    t = walled_box(size, size)
    c = size // 2
    t[c - 5:c + 5, size - 1] = EXIT
    return Scenario(f"room_{size}x{size}", t, n_agents, v, 1.2, seed, scn)


def _place_exits(t: np.ndarray, rng: np.random.Generator, count: int,
                 widths=None, centred: bool = False) -> list:
    H, W = t.shape
    exits = []
    sides = [0, 1, 2, 3] if centred else list(rng.integers(0, 4, size=count))
    for k in range(count):
        side = int(sides[k % len(sides)])
        width = int(widths[k]) if widths is not None else int(rng.integers(2, 11))
        length = (W if side in (0, 1) else H) - 2          # inner border length
        width = max(1, min(width, length))
        off = (length - width) // 2 if centred else int(rng.integers(0, length - width + 1))
        lo = 1 + off
        if side == 0:
            t[0, lo:lo + width] = EXIT
            exits.append((lo, 0, lo + width - 1, 0))
        elif side == 1:
            t[H - 1, lo:lo + width] = EXIT
            exits.append((lo, H - 1, lo + width - 1, H - 1))
        elif side == 2:
            t[lo:lo + width, 0] = EXIT
            exits.append((0, lo, 0, lo + width - 1))
        else:
            t[lo:lo + width, W - 1] = EXIT
            exits.append((W - 1, lo, W - 1, lo + width - 1))
    return exits


def _add_pillars(t: np.ndarray, rng: np.random.Generator, frac: float) -> None:
    """Random rectangles (sides 1..4) on free interior cells until the wall
    coverage of the interior reaches `frac`; no pillar comes within 2 cells of
    an exit cell."""
    H, W = t.shape
    interior = (H - 2) * (W - 2)
    if frac <= 0 or interior <= 0:
        return
    ey, ex = np.nonzero(t == EXIT)
    keep_out = np.zeros_like(t, dtype=bool)
    for y, x in zip(ey, ex):
        keep_out[max(0, y - 2):y + 3, max(0, x - 2):x + 3] = True
    target = int(np.ceil(frac * interior))
    covered = 0
    attempts = 0
    while covered < target and attempts < 50 * interior:
        attempts += 1
        h = int(rng.integers(1, 5))
        w = int(rng.integers(1, 5))
        y0 = int(rng.integers(1, max(2, H - 1 - h + 1)))
        x0 = int(rng.integers(1, max(2, W - 1 - w + 1)))
        y1, x1 = min(y0 + h, H - 1), min(x0 + w, W - 1)
        if keep_out[y0:y1, x0:x1].any():
            continue
        block = t[y0:y1, x0:x1]
        covered += int((block == FREE).sum())
        block[...] = WALL


def ensemble_member(k: int, base_seed: int = 2, scn_base: int = 0) -> Scenario:
    """Scenario k of the 256-member ensemble workload (also the distribution
    the serving workload draws its requests from)."""
    rng = np.random.default_rng([base_seed, k])
    W = int(rng.integers(30, 301))
    H = int(rng.integers(30, 301))
    frac = float(rng.uniform(0.0, 0.15))
    t = walled_box(W, H)
    n_exits = int(rng.integers(1, 5))
    _place_exits(t, rng, n_exits)
    _add_pillars(t, rng, frac)
    n_free = int((t == FREE).sum())
    n = int(round(float(np.exp(rng.uniform(np.log(50.0), np.log(20000.0))))))
    n = max(1, min(n, n_free // 2))
    v = int(rng.integers(1, 6))
    return Scenario(f"ensemble_{k}", t, n, v, 1.2, base_seed, scn_base + k,
                    meta={"pillar_frac": frac, "exits": n_exits})


def ensemble(count: int = 256, base_seed: int = 2) -> list:
    return [ensemble_member(k, base_seed) for k in range(count)]


def large_member(k: int, size: int = 1000, n_agents: int = 200000, base_seed: int = 3,
                 pillar_frac: float = 0.10) -> Scenario:
    rng = np.random.default_rng([base_seed, k])
    t = walled_box(size, size)
    _place_exits(t, rng, 4, widths=[10, 10, 10, 10], centred=True)
    _add_pillars(t, rng, pillar_frac)
    n_free = int((t == FREE).sum())
    n = min(n_agents, n_free // 2)
    return Scenario(f"large_{k}", t, n, 4, 1.2, base_seed, k)


def large(count: int = 16, **kw) -> list:
    return [large_member(k, **kw) for k in range(count)]


def random_small(rng: np.random.Generator, W: int, H: int, pillar_frac: float,
                 n_agents: int, v: int, k_s: float = 1.2, seed: int = 7,
                 scn: int = 0, n_exits: int = 1) -> Scenario:
    """Tiny random room used by the invariant and parity tests."""
    t = walled_box(W, H)
    _place_exits(t, rng, n_exits, widths=[int(rng.integers(1, 4)) for _ in range(n_exits)])
    _add_pillars(t, rng, pillar_frac)
    n_free = int((t == FREE).sum())
    return Scenario(f"small_{W}x{H}", t, min(n_agents, max(0, n_free // 2)), v, k_s, seed, scn)


def counterflow(n_agents: int = 300, v: int = 4, seed: int = 4, scn: int = 0, W: int = 60,
                H: int = 20) -> Scenario:
    """Two groups crossing a walled hall: exits in the middle of the left and
    the right wall; field 0 leads to the right exits, field 1 to the left
    ones.  meta: exit_field (H, W) uint8 (the field of each exit cell) and
    agent_field (n,) uint8, an even seeded mix of the two groups."""
    t = walled_box(W, H)
    c = H // 2
    t[c - 2:c + 2, W - 1] = EXIT
    t[c - 2:c + 2, 0] = EXIT
    ef = np.zeros((H, W), dtype=np.uint8)
    ef[c - 2:c + 2, 0] = 1
    rng = np.random.default_rng([seed, scn, 17])
    af = rng.permutation(np.arange(n_agents) % 2).astype(np.uint8)
    return Scenario(f"counterflow_{W}x{H}", t, n_agents, v, 1.2, seed, scn,
                    meta={"exit_field": ef, "agent_field": af})


CELL_M2 = 0.16                     # one 0.4 m x 0.4 m cell


def fd_corridor(density: float, scn: int, length: int = 100, width: int = 10, fill: int = 50,
                v: int = 4, seed: int = 5, exit_cells: int = 0) -> Scenario:
    """Corridor for a fundamental diagram at an initial `density` (persons
    per m^2) over the first `fill` columns.  Its right wall is the exit, or
    with exit_cells > 0 a bottleneck: only that many cells in the middle of
    it.  meta: agent_xy (n, 2), the rectangles `area` (measurement area, 10
    columns full width, from x = 61; with a bottleneck from x = 81, inside
    the queue in front of it) and `upstream` (every cell left of the line
    after the area's last column), area_m2 and width_m."""
    W, H = length + 2, width + 2
    t = walled_box(W, H)
    if exit_cells <= 0 or exit_cells >= width:
        t[1:H - 1, W - 1] = EXIT
    else:
        y0 = 1 + (width - exit_cells) // 2
        t[y0:y0 + exit_cells, W - 1] = EXIT
    n = min(int(round(density * fill * width * CELL_M2)), fill * width)
    rng = np.random.default_rng([seed, scn])
    cells = rng.choice(fill * width, size=n, replace=False)
    xy = np.stack([1 + cells % fill, 1 + cells // fill], axis=1).astype(np.int32)
    bottleneck = 0 < exit_cells < width
    a0 = length - 19 if bottleneck else 61
    meta = {"agent_xy": xy, "area": (a0, 1, a0 + 10, H - 1), "upstream": (0, 0, a0 + 10, H),
            "area_m2": 10 * width * CELL_M2, "width_m": width * 0.4, "density0": density,
            "exit_cells": exit_cells if bottleneck else width}
    name = f"fd_b{exit_cells}_{density:g}_{scn}" if bottleneck else f"fd_{density:g}_{scn}"
    return Scenario(name, t, n, v, 1.2, seed, scn, meta)


def fd_ensemble(densities=(0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 4.5, 5.0, 5.5),
                per_density: int = 16) -> list:
    """fd_corridor members: per_density seeds of each initial density,
    scenario ids 1000 * (density index) + k."""
    return [fd_corridor(d, 1000 * i + k) for i, d in enumerate(densities) for k in range(per_density)]


def fd_bottleneck_ensemble(exit_widths=(1, 2), densities=(4.0, 5.0, 6.0),
                           per_case: int = 16) -> list:
    """Bottleneck corridors for the congested branch: a queue builds up
    behind an exit narrower than the corridor and covers the measurement
    area in front of it, where the flow across the line is the bottleneck's
    outflow and the density that of the queue (in this model an exit cell
    removes agents as fast as they reach it, so exits of 3 cells and more
    already keep up with the corridor).  Scenario ids 50000 + 1000 *
    (width index) + 100 * (density index) + k."""
    return [fd_corridor(d, 50000 + 1000 * i + 100 * j + k, exit_cells=w)
            for i, w in enumerate(exit_widths) for j, d in enumerate(densities)
            for k in range(per_case)]
