"""Oracle pins of the dynamic floor field (reading R14), on the CPU.

The paper fixes k_other = 0 (Sec. 2) and cites the couplings without stating
them, so the trail field is a reading of this project: deposits by agents that
leave their cell, decay delta and diffusion alpha after every motion phase, a
weight factor exp(k_D (T(t) - T(c))).  These tests pin the oracle's
implementation to closed forms of that reading and to the static model it must
reduce to.
"""
import math

import numpy as np
import pytest

import oracle
from paper_0911_2900_amd import scenarios as sc


def _open_room(size=41):
    t = sc.walled_box(size, size)
    t[size // 2, size - 1] = oracle.CELL_EXIT
    return t


def test_k_d_zero_reproduces_the_static_model():
    """Trail bookkeeping with k_D = 0 changes no weight bit: every plan and
    every position equal the plain model's, step by step."""
    for s in (sc.room(size=60, n_agents=600, v=4), sc.ensemble_member(3), sc.corridor()):
        a = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
        b = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents,
                       trail=(0.0, 0.3, 0.2))
        for _ in range(25):
            a.plan()
            b.plan()
            assert np.array_equal(a.desired, b.desired)
            a.move()
            b.move()
            a.end_step()
            b.end_step()
            assert np.array_equal(a.positions(), b.positions())
        assert b.Tr.sum() > 0                      # the field was kept all along


def test_single_deposit_decays_geometrically():
    """alpha = 0: one deposit of 1 becomes exactly (1 - delta)^t after t
    further updates (delta = 1/4: every power of 3/4 up to t = 33 is exact in
    FP64), and no other cell ever holds anything."""
    t = _open_room()
    sim = oracle.Sim(t, 2, 1.2, 1, 0, n_agents=0, trail=(1.0, 0.25, 0.0))
    c = (20, 17)
    sim.dep[c] = 1
    sim.trail_update()
    assert sim.Tr[c] == 1.0 and sim.dep.sum() == 0
    for k in range(1, 34):
        sim.trail_update()
        assert sim.Tr[c] == 0.75 ** k, k
        assert np.count_nonzero(sim.Tr) == 1


def test_one_diffusion_step_from_a_point():
    """From T = 1 at one open cell: (1 - delta)(1 - alpha) stays, each of the
    8 neighbours gets (1 - delta) alpha / 8, nothing else."""
    t = _open_room()
    d, a = 0.5, 0.5
    sim = oracle.Sim(t, 2, 1.2, 1, 0, n_agents=0, trail=(1.0, d, a))
    sim.Tr[20, 20] = 1.0
    sim.trail_update()
    assert sim.Tr[20, 20] == (1 - d) * (1 - a)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx or dy:
                assert sim.Tr[20 + dy, 20 + dx] == (1 - d) * a / 8
    assert np.count_nonzero(sim.Tr) == 9


def test_diffusion_without_decay_conserves_mass_and_symmetry():
    """delta = 0, away from walls: the total stays the deposit (rounding
    only), and the spread keeps the 8 symmetries of the square grid."""
    t = _open_room(61)
    sim = oracle.Sim(t, 2, 1.2, 1, 0, n_agents=0, trail=(1.0, 0.0, 0.5))
    sim.dep[30, 30] = 1
    for _ in range(12):
        sim.trail_update()
        assert abs(sim.Tr.sum() - 1.0) < 1e-14
    w = sim.Tr[18:43, 18:43]
    for g in (w[::-1, :], w[:, ::-1], w.T, w[::-1, ::-1].T):
        assert np.allclose(g, w, rtol=1e-13, atol=0)


def test_walls_stay_empty_and_leak_nothing_back():
    t = _open_room(11)
    sim = oracle.Sim(t, 2, 1.2, 1, 0, n_agents=0, trail=(1.0, 0.1, 0.9))
    sim.dep[1, 1] = 5                              # next to the corner walls
    for _ in range(6):
        sim.trail_update()
        walls = sim.type == oracle.CELL_WALL
        assert np.all(sim.Tr[walls] == 0.0)
        assert np.all(sim.Tr >= 0.0)


def test_a_moving_agent_leaves_one_unit_at_its_start():
    """alpha = 0: after one step the trail is exactly 1 on the cell a single
    agent left (if it moved) and 0 everywhere else."""
    t = _open_room()
    moved = 0
    for seed in range(1, 30):
        sim = oracle.Sim(t, 3, 1.2, seed, 0, n_agents=1, trail=(0.5, 0.4, 0.0))
        x0, y0 = sim.x[0], sim.y[0]
        sim.step_once()
        if (sim.x[0], sim.y[0]) != (x0, y0):
            moved += 1
            assert sim.Tr[y0, x0] == 1.0
            assert np.count_nonzero(sim.Tr) == 1
        else:
            assert np.count_nonzero(sim.Tr) == 0
    assert moved > 10


@pytest.mark.parametrize("k_d", [0.7, 2.5])
def test_trail_weight_odds_ratio(k_d):
    """Two window cells at the same floor-field value: their weights are in
    the ratio exp(k_D (T1 - T2)); relative to the own cell, each weight is
    exp(k_S (S(c) - S(t)) + k_D (T(t) - T(c)))."""
    t = _open_room()
    sim = oracle.Sim(t, 2, 1.2, 1, 0, agent_xy=[[10, 20]], trail=(k_d, 0.2, 0.1))
    side = 5
    # cells (10, 18) and (10, 22) mirror each other about the exit row: same S
    sim.Tr[18, 10] = 1.75
    sim.Tr[22, 10] = 0.5
    sim.Tr[20, 10] = 0.25
    _, w, C, u, slot = sim.plan_agent(0)
    up, down = (0 * side + 2), (4 * side + 2)
    assert sim.S[18, 10] == sim.S[22, 10]
    assert math.isclose(w[up] / w[down], math.exp(k_d * (1.75 - 0.5)), rel_tol=1e-14)
    for sl in (up, down):
        dy = sl // side - 2
        ty = 20 + dy
        want = math.exp(1.2 * (sim.S[20, 10] - sim.S[ty, 10]) + k_d * (sim.Tr[ty, 10] - 0.25))
        assert w[sl] == want
