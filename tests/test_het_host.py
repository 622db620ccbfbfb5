"""Per-agent maximum speeds in the oracle (agent i reaches only its own disc
dx^2 + dy^2 <= v_i^2 inside the (2 v_max + 1)^2 window)."""
import numpy as np
import pytest

import oracle
from paper_0911_2900_amd import scenarios as sc


def _small(seed, v=4, n=200):
    rng = np.random.default_rng(seed)
    return sc.random_small(rng, 40, 30, 0.08, n, v, n_exits=2)


@pytest.mark.parametrize("seed", [0, 1])
def test_speeds_all_v_max_equal_the_uniform_model(seed):
    s = _small(seed)
    a = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents)
    b = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents,
                   agent_v=np.full(s.n_agents, s.v))
    for _ in range(25):
        a.step_once()
        b.step_once()
    assert np.array_equal(a.positions(), b.positions())
    assert a.exited == b.exited


@pytest.mark.parametrize("seed", [2, 3])
def test_every_plan_stays_in_the_agents_own_disc(seed):
    s = _small(seed, v=5, n=250)
    vi = np.random.default_rng(seed).integers(1, 6, size=s.n_agents)
    sim = oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents, agent_v=vi)
    W = sim.W
    for _ in range(20):
        sim.plan()
        alive = np.nonzero(sim.alive[: sim.n])[0]
        d = sim.desired[alive]
        dx = d % W - sim.x[alive]
        dy = d // W - sim.y[alive]
        assert (dx * dx + dy * dy <= vi[alive] * vi[alive]).all()
        sim.move()
        sim.end_step()


def test_weights_of_a_slow_agent_are_its_reachable_disc():
    """An agent of speed 2 among agents of v_max = 4: weights are
    exp(k_S (S(c) - S(t))) on the free cells of its radius-2 disc and zero
    everywhere else in the 9 x 9 window."""
    t = sc.walled_box(20, 20)
    t[8:12, 19] = sc.EXIT
    xy = np.array([[10, 10], [11, 10], [9, 12], [12, 13], [3, 3]], dtype=np.int32)
    vi = np.array([2, 4, 4, 4, 1])
    sim = oracle.Sim(t, 4, 1.2, 1, 0, agent_xy=xy, agent_v=vi)
    _, S = oracle.floor_field(t)[:2]
    occupied = {(int(x), int(y)) for x, y in xy}
    _, w, _, _, _ = sim.plan_agent(0)
    w = w.reshape(9, 9)
    for dy in range(-4, 5):
        for dx in range(-4, 5):
            x, y = 10 + dx, 10 + dy
            reach = (dx * dx + dy * dy <= 4 and t[y, x] != sc.WALL
                     and ((x, y) not in occupied or (dx, dy) == (0, 0)))
            if reach:       # libm and numpy exp may round differently: 2 ulp
                want = np.exp(1.2 * (S[10, 10] - S[y, x]))
                assert w[dy + 4, dx + 4] == pytest.approx(want, rel=4.5e-16, abs=0), (dx, dy)
            else:
                assert w[dy + 4, dx + 4] == 0.0, (dx, dy)
    # (11, 10) is taken by agent 1 and (9, 12) by agent 2: both inside the disc, weight 0
    assert w[4, 5] == 0.0 and w[6, 3] == 0.0


def test_bad_speeds_are_refused():
    s = _small(4, v=3, n=20)
    for bad in (np.full(s.n_agents, 4), np.zeros(s.n_agents), np.ones(s.n_agents - 1)):
        with pytest.raises(ValueError):
            oracle.Sim(s.cell_type, s.v, s.k_s, s.seed, s.scn, n_agents=s.n_agents, agent_v=bad)
