"""Several floor fields in the oracle (route choice, counterflow): agent i
weighs its window with the exact floor field of its own group's exits."""
import numpy as np
import pytest

import oracle
from paper_0911_2900_amd import scenarios as sc


def _corridor(W=12):
    t = np.ones((3, W), dtype=np.uint8)
    t[1, 1:W - 1] = 0
    t[1, 0] = 2
    t[1, W - 1] = 2
    ef = np.zeros_like(t)
    ef[1, W - 1] = 1
    return t, ef


def test_corridor_fields_are_the_distances_to_each_end():
    # one row between walls: field 0 counts cells from the left exit, field 1
    # from the right one, exactly (orthogonal steps only)
    W = 12
    t, ef = _corridor(W)
    after = oracle.floor_field(t)[0]
    x = np.arange(W, dtype=np.float64)
    assert np.array_equal(oracle.floor_field_of(after, ef, 0)[1], x)
    assert np.array_equal(oracle.floor_field_of(after, ef, 1)[1], W - 1 - x)
    assert np.all(np.isinf(oracle.floor_field_of(after, ef, 0)[0]))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_the_all_exit_field_is_the_minimum_of_the_group_fields(seed):
    # a shortest path from the union of the exit sets starts at one of them
    rng = np.random.default_rng(seed)
    s = sc.random_small(rng, 45, 35, 0.12, 0, 4, n_exits=4)
    after, S = oracle.floor_field(s.cell_type)[:2]
    ef = rng.integers(0, 3, size=after.shape).astype(np.uint8)
    for g in range(3):                      # every group owns at least one exit cell
        ef[np.argwhere(after == 2)[g][0], np.argwhere(after == 2)[g][1]] = g
    F = np.stack([oracle.floor_field_of(after, ef, g) for g in range(3)])
    open_ = after != 1
    assert np.array_equal(F.min(axis=0)[open_], S[open_])
    # exits of a group sit at 0 of their own field only where tagged
    for g in range(3):
        assert np.all(F[g][(after == 2) & (ef == g)] == 0)
        assert np.all(F[g][(after == 2) & (ef != g)] > 0)


def test_weights_follow_the_agents_own_field():
    # agents of opposite groups in the corridor: w(+1) / w(own) is e^{k} for
    # the group heading right and e^{-k} for the one heading left
    W, k = 12, 1.2
    t, ef = _corridor(W)
    sim = oracle.Sim(t, 1, k, 5, 0, agent_xy=[[3, 1], [8, 1]],
                     exit_field=ef, agent_field=[1, 0])
    _, w0, _, _, _ = sim.plan_agent(0)      # heads right (field 1)
    _, w1, _, _, _ = sim.plan_agent(1)      # heads left (field 0)
    # window 3x3, raster order; the row of the agent is slots 3, 4, 5
    assert w0[4] == 1.0 and w1[4] == 1.0
    assert w0[5] == pytest.approx(np.exp(k), rel=1e-15)
    assert w0[3] == pytest.approx(np.exp(-k), rel=1e-15)
    assert w1[5] == pytest.approx(np.exp(-k), rel=1e-15)
    assert w1[3] == pytest.approx(np.exp(k), rel=1e-15)
    assert np.all(w0[[0, 1, 2, 6, 7, 8]] == 0)


@pytest.mark.parametrize("seed", [0, 1])
def test_one_field_for_all_exits_equals_the_single_field_model(seed):
    rng = np.random.default_rng(seed)
    s = sc.random_small(rng, 40, 30, 0.08, 200, 4, n_exits=2)
    a = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    b = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents,
                   exit_field=np.zeros(s.cell_type.shape, np.uint8),
                   agent_field=np.zeros(s.n_agents, np.uint8))
    for _ in range(25):
        a.step_once()
        b.step_once()
    assert np.array_equal(a.positions(), b.positions())
    assert a.exited == b.exited


def test_counterflow_groups_leave_by_their_own_side():
    # with k_S = 1.2 nearly every agent ends at its own group's exit; count
    # the agents of each group that left through the far wall's column
    s = sc.counterflow(n_agents=120, v=3)
    ef, af = s.meta["exit_field"], s.meta["agent_field"]
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents,
                     exit_field=ef, agent_field=af)
    last = sim.positions().copy()
    for _ in range(200):
        sim.step_once()
        alive = sim.positions()[:, 0] >= 0
        last[alive] = sim.positions()[alive]
        if not alive.any():
            break
    assert sim.exited == s.n_agents
    # the last cell before leaving is next to the exit the agent used
    right = last[:, 0] > s.W // 2
    assert np.mean(right[af == 0]) > 0.95 and np.mean(~right[af == 1]) > 0.95


def _bellman_ford(after: np.ndarray, sources: np.ndarray) -> np.ndarray:
    """Shortest walking length from the source cells by repeated relaxation
    over the 8 neighbours (orthogonal 1, diagonal sqrt 2 when neither
    orthogonal neighbour is a wall); no priority queue, no exact lengths."""
    H, W = after.shape
    D = np.full((H, W), np.inf)
    D[sources] = 0.0
    wall = after == 1
    changed = True
    while changed:
        changed = False
        for y in range(H):
            for x in range(W):
                if wall[y, x]:
                    continue
                best = D[y, x]
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        ny, nx = y + dy, x + dx
                        if (dx == 0 and dy == 0) or not (0 <= ny < H and 0 <= nx < W) or wall[ny, nx]:
                            continue
                        if dx and dy:
                            if wall[y, nx] or wall[ny, x]:
                                continue
                            step = np.sqrt(2.0)
                        else:
                            step = 1.0
                        best = min(best, D[ny, nx] + step)
                if best < D[y, x]:
                    D[y, x] = best
                    changed = True
    return D


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_group_fields_equal_brute_force_relaxation(seed):
    rng = np.random.default_rng(seed)
    s = sc.random_small(rng, 14, 11, 0.15, 0, 3, n_exits=3)
    after = oracle.floor_field(s.cell_type)[0]
    exits = np.argwhere(after == 2)
    ef = np.zeros_like(after)
    ef[tuple(exits.T)] = rng.integers(0, 2, size=len(exits))
    ef[tuple(exits[0])] = 0
    ef[tuple(exits[-1])] = 1
    for g in (0, 1):
        F = oracle.floor_field_of(after, ef, g)
        B = _bellman_ford(after, (after == 2) & (ef == g))
        finite = np.isfinite(B)
        assert np.array_equal(finite, np.isfinite(F))
        assert np.allclose(F[finite], B[finite], rtol=0, atol=1e-12)
